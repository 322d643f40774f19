"""Pins for the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or the mathematics
fixes: hand-derived kernel values, closed forms, invariants, a library routine
in a special case, brute force on tiny inputs, and an independent exact lasso
solver.  The planted-mistake tests at the end show that plausible slips in the
oracle (a dropped term, a flipped sign, a transposed operand) fail these pins.
"""

import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import optimize

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers that are independent of the oracle
# ---------------------------------------------------------------------------

def load_kernel_fixture(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        lines = [l.strip() for l in f if l.strip() and not l.startswith("#")]
    hdr = lines[0].split()
    nx, ny = int(hdr[0]), int(hdr[1])
    b = tuple(float(v) for v in hdr[2:5])
    vox = (float(hdr[5]), float(hdr[6]))
    for l in lines[1:]:
        rows.append([float(Fraction(t)) for t in l.split()])
    D = np.array(rows)
    assert D.shape == (ny, nx)
    return nx, ny, b, vox, D


def dense_A_from_cosines(D):
    """Dense matrix of A on an ny x nx slice built from explicit cosine sums:
    A[r, r'] = 1/(nx ny) sum_k D(k) cos(2 pi (kx (x-x')/nx + ky (y-y')/ny)).
    Uses no DFT matrix, no FFT and no oracle code."""
    ny, nx = D.shape
    npix = nx * ny
    ys, xs = np.divmod(np.arange(npix), nx)
    A = np.zeros((npix, npix))
    for ky in range(ny):
        for kx in range(nx):
            if D[ky, kx] == 0.0:
                continue
            ph = 2.0 * np.pi * (kx * xs / nx + ky * ys / ny)
            c, s = np.cos(ph), np.sin(ph)
            # cos(a - b) = cos a cos b + sin a sin b
            A += D[ky, kx] * (np.outer(c, c) + np.outer(s, s))
    return A / npix


def lasso_exact(A, d, lam):
    """Lasso by a bound-constrained smooth QP (x = u - v, u, v >= 0) solved
    with L-BFGS-B: an algorithm unrelated to primal-dual splitting."""
    n = A.shape[1]

    def f(w):
        u, v = w[:n], w[n:]
        r = A @ (u - v) - d
        g = A.T @ r
        return 0.5 * r @ r + lam * np.sum(w), np.concatenate([g + lam, -g + lam])

    w0 = np.zeros(2 * n)
    res = optimize.minimize(f, w0, jac=True, method="L-BFGS-B",
                            bounds=[(0, None)] * (2 * n),
                            options=dict(maxiter=200000, ftol=1e-16, gtol=1e-13, maxcor=50))
    x = res.x[:n] - res.x[n:]
    return x, res.fun


def lasso_objective(A, d, lam, x):
    r = A @ x - d
    return 0.5 * r @ r + lam * np.sum(np.abs(x))


# ---------------------------------------------------------------------------
# frequency grid and DFT
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 64, 96, 192, 384])
@pytest.mark.parametrize("d", [1.0, 0.72])
def test_kgrid_is_numpy_fftfreq(n, d):
    np.testing.assert_allclose(O.kgrid(n, d), np.fft.fftfreq(n, d), rtol=0, atol=1e-15)


@pytest.mark.parametrize("shape", [(8, 8), (4, 12), (6, 10)])
def test_dft_impulse_is_all_ones(shape):
    x = np.zeros(shape)
    x[0, 0] = 1.0
    np.testing.assert_allclose(O.dft2(x), np.ones(shape), atol=1e-14)


@pytest.mark.parametrize("shape", [(8, 8), (6, 12), (9, 5)])
def test_dft_of_pure_exponential_is_spike(shape):
    ny, nx = shape
    ky0, kx0 = 2 % ny, 3 % nx
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = np.exp(2j * np.pi * (kx0 * xx / nx + ky0 * yy / ny))
    X = O.dft2(x)
    expect = np.zeros(shape, dtype=complex)
    expect[ky0, kx0] = nx * ny
    np.testing.assert_allclose(X, expect, atol=1e-11)


@pytest.mark.parametrize("shape", [(3, 16, 16), (2, 24, 12), (1, 5, 7)])
def test_dft_round_trip_and_parseval(shape):
    rng = np.random.default_rng(7)
    x = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    X = O.dft2(x)
    np.testing.assert_allclose(O.idft2(X), x, atol=1e-13)
    n = shape[-1] * shape[-2]
    np.testing.assert_allclose(np.sum(np.abs(X) ** 2) / n, np.sum(np.abs(x) ** 2), rtol=1e-13)


@pytest.mark.parametrize("shape", [(2, 64, 64), (1, 192, 96), (1, 384, 24)])
def test_dft_matches_library_fft(shape):
    rng = np.random.default_rng(3)
    x = rng.normal(size=shape)
    X = O.dft2(x)
    ref = np.fft.fft2(x)
    assert np.max(np.abs(X - ref)) <= 1e-10 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# dipole kernel
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["dipole_4x4_b0y.txt", "dipole_3x3_b0xy.txt",
                                  "dipole_4x2_b0z_aniso.txt"])
def test_dipole_kernel_hand_derived(name):
    nx, ny, b, vox, D = load_kernel_fixture(name)
    np.testing.assert_allclose(O.dipole_kernel(nx, ny, b, vox), D, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [8, 16, 64, 192, 256])
def test_dipole_range_origin_and_evenness(n):
    D = O.dipole_kernel(n, n, (0, 1, 0))
    assert D[0, 0] == 0.0
    assert D.min() == pytest.approx(-2.0 / 3.0, abs=1e-15)   # k along B0
    assert D.max() == pytest.approx(1.0 / 3.0, abs=1e-15)    # k perpendicular
    assert np.all(D >= -2.0 / 3.0 - 1e-15) and np.all(D <= 1.0 / 3.0 + 1e-15)
    neg = D[(-np.arange(n)) % n][:, (-np.arange(n)) % n]
    np.testing.assert_array_equal(D, neg)
    assert O.kernel_norm(D) == pytest.approx(2.0 / 3.0)


def test_dipole_even_with_oblique_b0_on_even_grid():
    D = O.dipole_kernel(8, 6, (0.6, 0.8, 0.0))
    neg = D[(-np.arange(6)) % 6][:, (-np.arange(8)) % 8]
    np.testing.assert_array_equal(D, neg)
    x = np.random.default_rng(0).normal(size=(1, 6, 8))
    O.apply_A(x, D)          # real to 1e-10 (asserted inside)


def test_dipole_voxel_scaling_only_rescales_axes():
    # doubling dx halves kx; the kernel at (kx/2, ky) equals the kernel on a grid
    # whose ky is doubled instead (D is homogeneous of degree 0 in k)
    D1 = O.dipole_kernel(8, 8, (0, 1, 0), (2.0, 1.0))
    D2 = O.dipole_kernel(8, 8, (0, 1, 0), (1.0, 0.5))
    np.testing.assert_allclose(D1, D2, atol=1e-15)


def test_dense_operator_from_cosines_matches_A_and_has_D_as_spectrum():
    D = O.dipole_kernel(8, 8, (0, 1, 0))
    A = dense_A_from_cosines(D)
    np.testing.assert_allclose(A, A.T, atol=1e-15)
    ev = np.sort(np.linalg.eigvalsh(A))
    np.testing.assert_allclose(ev, np.sort(D.ravel()), atol=1e-13)
    x = np.random.default_rng(5).normal(size=(3, 8, 8))
    ref = np.stack([(A @ s.ravel()).reshape(8, 8) for s in x])
    np.testing.assert_allclose(O.apply_A(x, D), ref, atol=1e-13)


def test_dense_operator_rectangular_oblique():
    D = O.dipole_kernel(6, 4, (0.3, 0.5, 0.8), (0.72, 1.0))
    A = dense_A_from_cosines(D)
    x = np.random.default_rng(6).normal(size=(2, 4, 6))
    ref = np.stack([(A @ s.ravel()).reshape(4, 6) for s in x])
    np.testing.assert_allclose(O.apply_A(x, D), ref, atol=1e-13)


# ---------------------------------------------------------------------------
# step-size validation
# ---------------------------------------------------------------------------

def test_step_validation():
    D = O.dipole_kernel(8, 8, (0, 1, 0))
    O.check_steps(1.4, 1.4, 1.0, D)                     # 1.96 * 4/9 = 0.871
    with pytest.raises(ValueError):
        O.check_steps(1.5, 1.5, 1.0, D)                 # exactly 1: the boundary
    with pytest.raises(ValueError):
        O.check_steps(1.4, 1.4, 1.5, D)
    with pytest.raises(ValueError):
        O.check_steps(-1.0, 1.0, 1.0, D)
    with pytest.raises(ValueError):
        O.dipole_kernel(8, 8, (0, 0, 0))


# ---------------------------------------------------------------------------
# proximal maps: brute-force minimisation of their defining objectives
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("v,t", [(2.0, 0.5), (-2.0, 0.5), (0.3, 0.5), (-0.5, 0.5),
                                 (0.5, 0.5), (1e-3, 1.4e-3), (7.0, 0.0)])
def test_prox_l1_bruteforce(v, t):
    res = optimize.minimize_scalar(lambda x: 0.5 * (x - v) ** 2 + t * abs(x),
                                   bounds=(-20, 20), method="bounded",
                                   options=dict(xatol=1e-12))
    assert O.prox_l1(v, t) == pytest.approx(res.x, abs=1e-8)


def test_prox_l1_exact_zero_inside_threshold():
    v = np.array([0.5, -0.5, 0.25, -0.0, 0.0])
    assert np.all(O.prox_l1(v, 0.5) == 0.0)


@pytest.mark.parametrize("w,delta,sigma", [(1.0, 0.3, 1.4), (-2.0, 1.0, 0.5), (0.0, -4.0, 2.0)])
def test_prox_dual_bruteforce(w, delta, sigma):
    # prox of sigma F*, F*(y) = 1/2 y^2 + y delta (conjugate of 1/2 (z - delta)^2)
    res = optimize.minimize_scalar(
        lambda y: sigma * (0.5 * y * y + y * delta) + 0.5 * (y - w) ** 2,
        bounds=(-50, 50), method="bounded", options=dict(xatol=1e-12))
    assert O.prox_dual(w, delta, sigma) == pytest.approx(res.x, abs=1e-8)


def test_conjugate_of_data_term_is_what_prox_dual_uses():
    # F(z) = 1/2 (z - delta)^2  =>  F*(y) = sup_z y z - F(z) = 1/2 y^2 + y delta
    delta = 0.7
    for y in (-1.3, 0.0, 2.2):
        res = optimize.minimize_scalar(lambda z: -(y * z - 0.5 * (z - delta) ** 2))
        assert -res.fun == pytest.approx(0.5 * y * y + y * delta, abs=1e-10)


# ---------------------------------------------------------------------------
# whole iteration
# ---------------------------------------------------------------------------

def dense_pd(A, d, lam, tau, sigma, theta, iters):
    """Primal-dual iteration on a dense operator (independent of the DFT)."""
    x = np.zeros_like(d)
    y = np.zeros_like(d)
    xb = x.copy()
    for _ in range(iters):
        y = (y + sigma * (A @ xb - d)) / (1 + sigma)
        v = x - tau * (A @ y)
        xn = np.sign(v) * np.maximum(np.abs(v) - tau * lam, 0)
        xb = xn + theta * (xn - x)
        x = xn
    return x


@pytest.mark.parametrize("b0,kind", [((0, 1, 0), "dipole"), ((0.3, 0.5, 0.8), "dipole")])
def test_dft_pd_equals_dense_matrix_pd(b0, kind):
    rng = np.random.default_rng(11)
    d = rng.normal(size=(2, 8, 8))
    D = O.dipole_kernel(8, 8, b0)
    A = dense_A_from_cosines(D)
    chi, info = O.solve(d, lam=0.1, tau=1.2, sigma=1.2, theta=1.0, max_iter=200, b0=b0)
    ref = np.stack([dense_pd(A, s.ravel(), 0.1, 1.2, 1.2, 1.0, 200).reshape(8, 8) for s in d])
    np.testing.assert_allclose(chi, ref, atol=1e-12)
    assert info["iterations"] == 200


def test_identity_kernel_converges_to_soft_threshold():
    # A = I: argmin 1/2||x - d||^2 + lam||x||_1 is soft(d, lam) in closed form
    rng = np.random.default_rng(2)
    d = rng.normal(size=(3, 8, 8))
    lam = 0.3
    chi, info = O.solve(d, lam=lam, tau=0.9, sigma=0.9, max_iter=400, kind="identity")
    closed = np.where(np.abs(d) > lam, d - lam * np.sign(d), 0.0)
    np.testing.assert_allclose(chi, closed, atol=1e-12)
    assert info["rel_gap"] < 1e-12


def test_identity_kernel_stops_on_gap_tolerance():
    rng = np.random.default_rng(4)
    d = rng.normal(size=(2, 8, 8))
    hist = []
    chi, info = O.solve(d, lam=0.2, tau=0.9, sigma=0.9, max_iter=1000, gap_tol=1e-8,
                        check_every=5, kind="identity", history=hist)
    assert info["iterations"] < 1000 and info["iterations"] % 5 == 0
    assert info["rel_gap"] <= 1e-8
    assert all(h[3] > 1e-8 for h in hist[:-1])     # stopped at the first passing check


def test_pd_reaches_exact_lasso_minimum_8x8():
    rng = np.random.default_rng(8)
    d = rng.normal(size=(8, 8))
    lam = 0.1
    D = O.dipole_kernel(8, 8, (0, 1, 0))
    A = dense_A_from_cosines(D)
    x_star, _ = lasso_exact(A, d.ravel(), lam)
    p_star = lasso_objective(A, d.ravel(), lam, x_star)
    # KKT certificate for the independent solution
    g = A.T @ (d.ravel() - A @ x_star)
    on = np.abs(x_star) > 1e-9
    assert np.max(np.abs(g[on] - lam * np.sign(x_star[on]))) < 1e-6
    assert np.max(np.abs(g[~on])) <= lam + 1e-6
    chi, info = O.solve(d[None], lam=lam, max_iter=5000)
    p_pd = lasso_objective(A, d.ravel(), lam, chi[0].ravel())
    assert p_pd == pytest.approx(p_star, rel=1e-9)
    assert info["primal"] == pytest.approx(p_star, rel=1e-9)
    assert 0.0 <= info["rel_gap"] < 1e-8
    # A chi is unique at the optimum even where chi is not
    np.testing.assert_allclose(A @ chi[0].ravel(), A @ x_star, atol=1e-5)


def test_weak_duality_and_geometric_gap_decrease():
    rng = np.random.default_rng(9)
    chi_true = np.zeros((1, 32, 32))
    yy, xx = np.mgrid[:32, :32]
    chi_true[0][(yy - 16) ** 2 + (xx - 16) ** 2 <= 4] = 180.0
    chi_true[0] += rng.normal(0, 0.05, size=(32, 32)) * ((yy - 16) ** 2 + (xx - 16) ** 2 > 4)
    field = O.forward(chi_true)
    d = field + 0.01 * np.abs(field).max() * rng.normal(size=field.shape)
    gaps = {}
    for n in (16, 32, 64, 128, 256, 512):
        _, info = O.solve(d, lam=1e-3, max_iter=n)
        assert info["primal"] - info["dual"] >= -1e-12 * info["primal"]
        gaps[n] = info["primal"] - info["dual"]
    vals = [gaps[n] for n in sorted(gaps)]
    assert all(b <= a for a, b in zip(vals, vals[1:])), vals


def test_zero_iterations_and_zero_field():
    d = np.zeros((1, 8, 8))
    chi, info = O.solve(d, lam=0.1, max_iter=0)
    assert info["iterations"] == 0 and np.all(chi == 0)
    chi, info = O.solve(d, lam=0.1, max_iter=50)
    assert np.all(chi == 0) and info["primal"] == 0.0 and info["dual"] == 0.0


def test_nonfinite_input_is_reported():
    d = np.zeros((1, 8, 8))
    d[0, 3, 3] = np.nan
    _, info = O.solve(d, lam=0.1, max_iter=20, gap_tol=1e-6, check_every=5)
    assert info["status"] == "nonfinite"


def test_solve_is_per_slice_independent_in_fixed_count_mode():
    rng = np.random.default_rng(12)
    d = rng.normal(size=(3, 16, 8))
    chi, _ = O.solve(d, lam=0.05, max_iter=60)
    for z in range(3):
        c1, _ = O.solve(d[z:z + 1], lam=0.05, max_iter=60)
        np.testing.assert_array_equal(chi[z], c1[0])


# ---------------------------------------------------------------------------
# planted mistakes: the pins above must catch plausible slips in the oracle
# ---------------------------------------------------------------------------

def _lasso_pin_passes():
    try:
        test_pd_reaches_exact_lasso_minimum_8x8()
        return True
    except AssertionError:
        return False


def _dense_pin_passes():
    try:
        test_dft_pd_equals_dense_matrix_pd((0.3, 0.5, 0.8), "dipole")
        return True
    except AssertionError:
        return False


def _plant(monkeypatch, name, fn):
    monkeypatch.setattr(O.pd_oracle, name, fn)
    monkeypatch.setattr(O, name, fn)


def test_planted_dropped_delta_term_is_caught(monkeypatch):
    _plant(monkeypatch, "prox_dual", lambda w, delta, sigma: w / (1.0 + sigma))
    assert not _lasso_pin_passes()


def test_planted_wrong_threshold_sign_is_caught(monkeypatch):
    good = O.pd_oracle.prox_l1
    _plant(monkeypatch, "prox_l1", lambda v, t: good(v, -t))
    assert not _lasso_pin_passes()


def test_planted_missing_overrelaxation_is_caught(monkeypatch):
    # theta silently ignored (chibar = chi): converges elsewhere / slower
    good = O.pd_oracle.solve

    def bad(delta, lam, tau=1.4, sigma=1.4, theta=1.0, **kw):
        return good(delta, lam, tau=tau, sigma=sigma, theta=0.0, **kw)
    _plant(monkeypatch, "solve", bad)
    assert not _dense_pin_passes()


def test_planted_flipped_dft_axis_is_caught(monkeypatch):
    good = O.pd_oracle.dft_matrix

    def bad_dft2(x):
        x = np.asarray(x)
        Wy = good(x.shape[-2])
        Wx = good(x.shape[-1], inverse=True)      # wrong sign along x
        return np.matmul(np.matmul(Wy, x.astype(np.complex128)), Wx.T)
    _plant(monkeypatch, "dft2", bad_dft2)
    assert not _dense_pin_passes()


def test_planted_swapped_kernel_axes_is_caught(monkeypatch):
    good = O.pd_oracle.dipole_kernel
    _plant(monkeypatch, "dipole_kernel",
           lambda nx, ny, b0=(0, 1, 0), voxel=(1, 1), kind="dipole":
           good(ny, nx, b0, voxel, kind).T.copy())
    with pytest.raises(AssertionError):
        test_dipole_kernel_hand_derived("dipole_4x4_b0y.txt")


def test_planted_kernel_without_origin_zero_is_caught(monkeypatch):
    good = O.pd_oracle.dipole_kernel

    def bad(nx, ny, b0=(0, 1, 0), voxel=(1, 1), kind="dipole"):
        D = good(nx, ny, b0, voxel, kind)
        D[0, 0] = 1.0 / 3.0
        return D
    _plant(monkeypatch, "dipole_kernel", bad)
    with pytest.raises(AssertionError):
        test_dipole_range_origin_and_evenness(16)


# ---------------------------------------------------------------------------
# 3-D kernel (whole-volume operator)
# ---------------------------------------------------------------------------

def load_kernel3_fixture(name):
    with open(os.path.join(GOLDEN, name)) as f:
        lines = [l.strip() for l in f if l.strip() and not l.startswith("#")]
    hdr = lines[0].split()
    nx, ny, nz = int(hdr[0]), int(hdr[1]), int(hdr[2])
    b = tuple(float(v) for v in hdr[3:6])
    vox = (float(hdr[6]), float(hdr[7]))
    dz = float(hdr[8])
    vals = [[float(Fraction(t)) for t in l.split()] for l in lines[1:]]
    D = np.array(vals).reshape(nz, ny, nx)
    return nx, ny, nz, b, vox, dz, D


@pytest.mark.parametrize("name", ["dipole3d_2x2x2_b0z.txt", "dipole3d_2x2x2_b0xy.txt",
                                  "dipole3d_3x1x2_b0z_dz2.txt"])
def test_dipole3d_kernel_hand_derived(name):
    nx, ny, nz, b, vox, dz, D = load_kernel3_fixture(name)
    np.testing.assert_allclose(O.dipole_kernel3(nx, ny, nz, b, vox, dz), D, atol=1e-15)


@pytest.mark.parametrize("b0", [(0, 1, 0), (0.3, 0.5, 0.8), (1, 0, 1)])
def test_dipole3d_kz0_plane_is_the_2d_kernel(b0):
    D3 = O.dipole_kernel3(12, 8, 6, b0, (0.8, 1.1), 2.0)
    np.testing.assert_allclose(D3[0], O.dipole_kernel(12, 8, b0, (0.8, 1.1)), atol=1e-15)


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 7), (8, 8, 8)])
def test_dipole3d_range_origin_and_evenness(shape):
    nz, ny, nx = shape
    D = O.dipole_kernel3(nx, ny, nz, (0.2, 0.7, 0.4), (1.0, 0.9), 1.5)
    assert D[0, 0, 0] == 0.0
    assert D.min() >= -2.0 / 3.0 - 1e-15 and D.max() <= 1.0 / 3.0 + 1e-15
    neg = D[(-np.arange(nz)) % nz][:, (-np.arange(ny)) % ny][:, :, (-np.arange(nx)) % nx]
    np.testing.assert_allclose(D, neg, atol=1e-15)


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 7)])
def test_dft3_round_trip_parseval_and_library(shape):
    rng = np.random.default_rng(8)
    x = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    X = O.dft3(x)
    np.testing.assert_allclose(X, np.fft.fftn(x), atol=1e-11)
    np.testing.assert_allclose(O.idft3(X), x, atol=1e-13)
    n = np.prod(shape)
    np.testing.assert_allclose(np.sum(np.abs(X) ** 2) / n, np.sum(np.abs(x) ** 2), rtol=1e-13)


def dense_A3_from_cosines(D):
    """Dense A on an nz x ny x nx volume from explicit cosine sums."""
    nz, ny, nx = D.shape
    n = nx * ny * nz
    idx = np.arange(n)
    zs, rem = np.divmod(idx, nx * ny)
    ys, xs = np.divmod(rem, nx)
    A = np.zeros((n, n))
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                if D[kz, ky, kx] == 0.0:
                    continue
                ph = 2.0 * np.pi * (kx * xs / nx + ky * ys / ny + kz * zs / nz)
                c, s = np.cos(ph), np.sin(ph)
                A += D[kz, ky, kx] * (np.outer(c, c) + np.outer(s, s))
    return A / n


def test_dense_3d_operator_matches_apply_A3():
    D = O.dipole_kernel3(4, 3, 2, (0.3, 0.5, 0.8), (1.0, 0.8), 1.6)
    A = dense_A3_from_cosines(D)
    np.testing.assert_allclose(A, A.T, atol=1e-14)
    rng = np.random.default_rng(9)
    x = rng.normal(size=(2, 3, 4))
    np.testing.assert_allclose(O.apply_A3(x, D).ravel(), A @ x.ravel(), atol=1e-13)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(D.ravel()), atol=1e-12)


def test_3d_operator_on_z_constant_volume_is_the_slice_operator():
    # a volume constant along z has only kz = 0 content, where D3 = D2
    rng = np.random.default_rng(10)
    sl = rng.normal(size=(6, 8))
    x = np.broadcast_to(sl, (4, 6, 8)).copy()
    a3 = O.forward(x, b0=(0.3, 0.5, 0.8), kind="dipole3d", voxel_z=2.0)
    a2 = O.forward(x, b0=(0.3, 0.5, 0.8))
    np.testing.assert_allclose(a3, a2, atol=1e-12)


def test_3d_pd_equals_dense_matrix_pd():
    D = O.dipole_kernel3(4, 3, 2, (0.3, 0.5, 0.8), (1.0, 0.8), 1.6)
    A = dense_A3_from_cosines(D)
    rng = np.random.default_rng(11)
    d = rng.normal(size=(2, 3, 4)) * 2
    lam, tau, sigma, theta = 0.05, 1.4, 1.4, 1.0
    ref = dense_pd(A, d.ravel(), lam, tau, sigma, theta, 40)
    chi, _ = O.solve(d, lam, tau, sigma, theta, 40, b0=(0.3, 0.5, 0.8), voxel=(1.0, 0.8), kind="dipole3d",
                     voxel_z=1.6)
    np.testing.assert_allclose(chi.ravel(), ref, atol=1e-11)


def test_planted_ignored_slice_thickness_is_caught(monkeypatch):
    good = O.pd_oracle.dipole_kernel3
    _plant(monkeypatch, "dipole_kernel3",
           lambda nx, ny, nz, b0=(0, 1, 0), voxel=(1, 1), voxel_z=1.0: good(nx, ny, nz, b0, voxel, 1.0))
    with pytest.raises(AssertionError):
        test_dipole3d_kernel_hand_derived("dipole3d_3x1x2_b0z_dz2.txt")


def dense_pd_with_dual(A, d, lam, tau, sigma, theta, iters):
    """dense_pd, also returning the dual iterate y_n."""
    x = np.zeros_like(d)
    y = np.zeros_like(d)
    xb = x.copy()
    for _ in range(iters):
        y = (y + sigma * (A @ xb - d)) / (1 + sigma)
        v = x - tau * (A @ y)
        xn = np.sign(v) * np.maximum(np.abs(v) - tau * lam, 0)
        xb = xn + theta * (xn - x)
        x = xn
    return x, y


def gap_from_definition(A, d, lam, x, y):
    """Primal objective, rescaled dual objective and relative gap written out
    from their definitions on a dense operator: P = 1/2||A x - d||^2 +
    lam||x||_1; s = min(1, lam / ||A y||_inf) makes s y dual-feasible for
    max -1/2||y||^2 - <y, d> s.t. ||A y||_inf <= lam."""
    r = A @ x - d
    P = 0.5 * r @ r + lam * np.sum(np.abs(x))
    m = np.max(np.abs(A @ y))
    s = 1.0 if m == 0 else min(1.0, lam / m)
    Dual = -0.5 * s * s * (y @ y) - s * (y @ d)
    return P, Dual, (P - Dual) / max(P, 1e-300)


@pytest.mark.parametrize("iters", [1, 7, 40])
def test_3d_objective_and_gap_equal_their_dense_definitions(iters):
    """The 3-D kernel's primal, dual and gap, pinned to a dense A3 from cosine
    sums and the gap's definition (no DFT, no oracle code): a gap evaluated
    with the slice-wise operator, a dropped term or a wrong scale fails."""
    b0, vox, dz = (0.3, 0.5, 0.8), (1.0, 0.8), 1.6
    D = O.dipole_kernel3(4, 3, 2, b0, vox, dz)
    A = dense_A3_from_cosines(D)
    rng = np.random.default_rng(12 + iters)
    d = rng.normal(size=(2, 3, 4)) * 2
    lam, tau, sigma, theta = 0.05, 1.4, 1.4, 1.0
    x, y = dense_pd_with_dual(A, d.ravel(), lam, tau, sigma, theta, iters)
    P, Dual, rel = gap_from_definition(A, d.ravel(), lam, x, y)
    _, info = O.solve(d, lam, tau, sigma, theta, iters, b0=b0, voxel=vox, kind="dipole3d", voxel_z=dz)
    assert info["primal"] == pytest.approx(P, rel=1e-12)
    assert info["dual"] == pytest.approx(Dual, rel=1e-11, abs=1e-13)
    assert info["rel_gap"] == pytest.approx(rel, rel=1e-10, abs=1e-13)
    # the same numbers from the gap-checked run (checks every iteration)
    _, info2 = O.solve(d, lam, tau, sigma, theta, iters, gap_tol=1e-300, check_every=1, b0=b0, voxel=vox,
                       kind="dipole3d", voxel_z=dz)
    assert info2["iterations"] == iters
    assert info2["primal"] == pytest.approx(P, rel=1e-12)
    assert info2["rel_gap"] == pytest.approx(rel, rel=1e-10, abs=1e-13)


def test_3d_pd_reaches_exact_lasso_minimum_4x3x2():
    """Converged 3-D solve against an independent lasso solver (L-BFGS-B on
    the dense A3) whose optimality is certified by the KKT conditions: the
    oracle's objective reaches the certified minimum and its gap closes."""
    b0, vox, dz = (0.3, 0.5, 0.8), (1.0, 0.8), 1.6
    D = O.dipole_kernel3(4, 3, 2, b0, vox, dz)
    A = dense_A3_from_cosines(D)
    rng = np.random.default_rng(13)
    d = rng.normal(size=(2, 3, 4))
    lam = 0.1
    x_star, _ = lasso_exact(A, d.ravel(), lam)
    p_star = lasso_objective(A, d.ravel(), lam, x_star)
    g = A.T @ (d.ravel() - A @ x_star)
    on = np.abs(x_star) > 1e-9
    assert on.any()
    assert np.max(np.abs(g[on] - lam * np.sign(x_star[on]))) < 1e-6
    assert np.max(np.abs(g[~on])) <= lam - 1e-3          # strictly feasible off the support
    chi, info = O.solve(d, lam=lam, max_iter=5000, b0=b0, voxel=vox, kind="dipole3d", voxel_z=dz)
    assert lasso_objective(A, d.ravel(), lam, chi.ravel()) == pytest.approx(p_star, rel=1e-9)
    assert info["primal"] == pytest.approx(p_star, rel=1e-9)
    assert 0.0 <= info["rel_gap"] < 1e-8
    np.testing.assert_allclose(A @ chi.ravel(), A @ x_star, atol=1e-5)


def test_planted_slicewise_operator_in_3d_gap_is_caught(monkeypatch):
    good = O.pd_oracle.duality_gap
    # the gap evaluated with the slice-wise operator instead of the 3-D one
    _plant(monkeypatch, "duality_gap", lambda chi, y, Ay, delta, D, lam, A=None: good(chi, y, Ay, delta, D, lam))
    with pytest.raises(AssertionError):
        test_3d_objective_and_gap_equal_their_dense_definitions(7)


def test_planted_unscaled_dual_in_gap_is_caught(monkeypatch):
    good = O.pd_oracle.duality_gap

    def no_rescale(chi, y, Ay, delta, D, lam, A=None):
        # the dual objective without the feasibility rescaling s
        P, _, _ = good(chi, y, Ay, delta, D, lam, A)
        Dual = -0.5 * float(np.sum(y * y)) - float(np.sum(y * delta))
        return P, Dual, (P - Dual) / max(P, 1e-300)
    _plant(monkeypatch, "duality_gap", no_rescale)
    with pytest.raises(AssertionError):
        test_3d_objective_and_gap_equal_their_dense_definitions(40)

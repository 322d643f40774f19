"""The seeded phantom generator: determinism and the stated distributions."""
import numpy as np

import pd_inputs as P


def test_seeded_and_deterministic():
    a, b = P.config2(nz=3), P.config2(nz=3)
    np.testing.assert_array_equal(a.chi_true, b.chi_true)
    np.testing.assert_array_equal(a.eta, b.eta)
    c = P.config2(seed=2001, nz=3)
    assert not np.array_equal(a.chi_true, c.chi_true)


def test_config1_disc():
    w = P.config1()
    assert w.shape == (1, 64, 64) and w.max_iter == 200 and w.lam == 1e-3
    yy, xx = np.mgrid[:64, :64]
    disc = (yy - 32) ** 2 + (xx - 32) ** 2 <= 9
    assert np.all(w.chi_true[0][disc] == 180.0)
    bg = w.chi_true[0][~disc]
    assert abs(bg.std() - P.TISSUE_SD) < 0.01 and abs(bg.mean()) < 0.01


def test_device_stack_values():
    w = P.config2(nz=6)
    vals = w.chi_true[w.chi_true > 1.0]
    assert np.all((vals == 100.0) | ((vals >= 150.0) & (vals <= 200.0)))
    for z in range(6):
        assert np.any(w.chi_true[z] >= 150.0)          # every slice has a needle


def test_tilted_needle_drifts_in_y():
    w = P.config4(nz=16)
    cy = [np.mean(np.nonzero(w.chi_true[z] == 180.0)[0]) for z in range(16)]
    steps = np.diff(cy)
    assert np.all(steps > 1.0)                          # ~ cot(30 deg) = 1.73 per slice
    assert abs(np.mean(steps) - np.sqrt(3.0)) < 0.2


def test_make_delta_scales_noise():
    field = np.array([[[0.0, -2.0], [1.0, 0.5]]])
    eta = np.ones_like(field)
    np.testing.assert_allclose(P.make_delta(field, eta, 0.01), field + 0.02)


def test_serving_schedule():
    s = P.serving_schedule()
    ts = [r[0] for r in s]
    assert all(0 < a < b < 60.0 for a, b in zip(ts, ts[1:]))
    assert 1000 < len(s) < 1400                        # 20/s for 60 s
    assert {r[1] for r in s} == set(P.SERVING_SIZES)
    assert min(r[2] for r in s) >= 16 and max(r[2] for r in s) <= 64


def test_serving_requests_drawn_on_the_gpu_follow_the_stack_recipe():
    """The per-request geometry of the GPU-drawn serving inputs is the one
    device_slice draws from the same generator state, slice by slice."""
    from pd_inputs.phantoms import device_objects, device_slice
    for seed in range(4):
        nz, ny, nx = 5, 48, 64
        z, y, x, v = device_objects(np.random.default_rng(seed), nz, ny, nx)
        rng = np.random.default_rng(seed)
        got = np.zeros((nz, ny, nx))
        cov = np.zeros((nz, ny, nx), dtype=bool)
        for a, b, c, d in zip(z, y, x, v):
            got[a, b, c] = d
            cov[a, b, c] = True
        for k in range(nz):
            val, c = device_slice(rng, ny, nx)
            assert np.array_equal(cov[k], c)
            assert np.array_equal(got[k][c], val[c])

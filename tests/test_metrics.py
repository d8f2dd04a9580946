"""Pins of the recovery metric of Section 6 (eq. (equ_MedSAE)) on the CPU.

The angles are built in by construction (each estimate is its original
component turned by a chosen angle in a chosen plane, then rescaled by a
signed factor and shuffled), so the metric is checked against the angle
itself, not against a second evaluation of its formula."""
import numpy as np

import cpgen
from paper_1205_2584_amd import metrics


def _turned(rng, a, theta):
    """Columns of a turned by the angles theta within random planes."""
    out = np.empty_like(a)
    for r in range(a.shape[1]):
        u = a[:, r] / np.linalg.norm(a[:, r])
        w = rng.standard_normal(a.shape[0]).astype(a.dtype)
        w -= u * np.vdot(u, w)
        w /= np.linalg.norm(w)
        out[:, r] = np.linalg.norm(a[:, r]) * (np.cos(theta[r]) * u + np.sin(theta[r]) * w)
    return out


def _estimate(rng, truth, thetas, perm, complex_=False):
    est = []
    for a, th in zip(truth, thetas):
        b = _turned(rng, a, th)
        scale = rng.uniform(0.2, 5.0, a.shape[1]) * rng.choice([-1.0, 1.0], a.shape[1])
        if complex_:
            scale = scale * np.exp(1j * rng.uniform(0, 2 * np.pi, a.shape[1]))
        est.append((b * scale)[:, perm])
    return est


def test_angles_recovered_through_order_sign_and_scale():
    rng = np.random.default_rng(0)
    for N, R, I in [(3, 5, 12), (4, 3, 7), (3, 8, 30)]:
        truth = [rng.standard_normal((I, R)) for _ in range(N)]
        thetas = [rng.uniform(1e-3, 0.3, R) for _ in range(N)]
        perm = rng.permutation(R)
        est = _estimate(rng, truth, thetas, perm)
        inv = np.argsort(perm)
        assert np.array_equal(metrics.match_order(truth, est), inv)
        a2 = metrics.squared_angular_errors(truth, est)
        assert a2.shape == (N, R)
        assert np.allclose(np.sqrt(a2), np.stack(thetas), rtol=1e-10, atol=0)


def test_tiny_angles_keep_their_accuracy():
    """1e-9 rad is below what arccos of a rounded cosine can resolve (about 1.5e-8)."""
    rng = np.random.default_rng(1)
    truth = [rng.standard_normal((40, 4)) for _ in range(3)]
    thetas = [np.full(4, 1e-9), np.full(4, 3e-10), np.array([1e-9, 2e-9, 0.1, 1e-7])]
    est = _estimate(rng, truth, thetas, np.arange(4))
    a2 = metrics.squared_angular_errors(truth, est)
    assert np.allclose(np.sqrt(a2), np.stack(thetas), rtol=1e-6, atol=0)


def test_complex_components_and_phase():
    rng = np.random.default_rng(2)
    truth = [rng.standard_normal((10, 3)) + 1j * rng.standard_normal((10, 3)) for _ in range(3)]
    thetas = [np.array([0.05, 0.2, 0.01])] * 3
    perm = np.array([2, 0, 1])
    est = _estimate(rng, truth, thetas, perm, complex_=True)
    a2 = metrics.squared_angular_errors(truth, est)
    assert np.allclose(np.sqrt(a2), np.stack(thetas), rtol=1e-10)


def test_medsae_median_and_decibels():
    # 3 runs x 1 mode x 2 components; medians 1e-3 and 4e-2
    runs = np.array([[[1e-4, 4e-2]], [[1e-2, 1.0]], [[1e-3, 1e-5]]])
    db = metrics.medsae_db(runs)
    assert np.allclose(db, [[-30.0, 10 * np.log10(4e-2)]], atol=1e-12)
    s = metrics.medsae_summary(runs)
    assert abs(s["medsae_first_db"] + 30.0) < 1e-12
    # angle scale printed with the metric: -30, -26 and -20 dB sit just below
    # angles of 2, 3 and 6 degrees
    for dbv, deg in [(-30.0, 2.0), (-26.0, 3.0), (-20.0, 6.0)]:
        ang = np.degrees(np.sqrt(10 ** (dbv / 10)))
        assert deg - 0.5 < ang < deg
    assert metrics.medsae_db(np.zeros((3, 1, 1)))[0, 0] == metrics.MEDSAE_FLOOR_DB


def test_exact_truth_matches_collinear_generator():
    """Collinear factors of the Section 6 generator (angles of 27 and 37 degrees
    at nu = 0.5) compared with themselves, shuffled and rescaled: every angle is
    zero to rounding and the order is recovered despite the collinearity."""
    rng = np.random.default_rng(3)
    A, _ = cpgen.nu_collinear_factors(rng, [30, 30, 30], 6, 0.5)
    perm = rng.permutation(6)
    est = _estimate(rng, A, [np.zeros(6)] * 3, perm)
    assert np.array_equal(metrics.match_order(A, est), np.argsort(perm))
    assert np.max(metrics.squared_angular_errors(A, est)) < 1e-28

"""Pins of the FP64 oracle against the paper and the mathematics (CPU only).

Each test checks the oracle against something other than itself: the plain
damped Gauss-Newton step with an explicitly formed Jacobian (Section 3,
Lemma B.1), closed forms (Theorem E.1, Appendix F), special cases (zero
gradient at an exact rank-R tensor, mu -> infinity), printed values
(Section 6 angle table, Section 4.3 densities) and brute-force loops.
Planted-mistake tests show that plausible errors in the oracle fail a pin.
"""
import json
import os

import numpy as np
import pytest

import cpgen
from oracle import brute, cp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SHAPES = [
    ((4, 3, 5), 1), ((5, 4, 3), 2), ((3, 5, 4), 3), ((4, 4, 4), 4),
    ((3, 4, 3, 4), 2), ((4, 3, 3, 3), 3), ((3, 3, 3, 3, 3), 2),
]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _problem(seed, dims, R, complex_=False, snr=20.0, c=0.4):
    p = cpgen.small_problem(seed, dims, R, c=c, snr_db=snr, complex_=complex_)
    return p, cp.as_tensor(p.y, dims)


@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("variant", ["a", "b"])
@pytest.mark.parametrize("mu", [1e-2, 1.0, 50.0])
@pytest.mark.parametrize("shape", SHAPES)
def test_fast_step_equals_explicit_solve(shape, mu, variant, complex_):
    dims, R = shape
    p, Y = _problem(11 + len(dims) * 7 + R, dims, R, complex_)
    st = cp.fast_step(Y, p.init, mu, variant=variant)
    da, g, _ = brute.plain_step(p.y, p.init, mu)
    assert _rel(cp.flat(st.dA), cp.flat(da)) < 1e-9
    assert _rel(cp.flat(st.g), g) < 1e-12


@pytest.mark.parametrize("complex_", [False, True])
def test_printed_w_simplification_fails(complex_):
    """Planted reading: w with the all-mode Hadamard Gamma (as printed in
    Theorem 4.1) does not reproduce the explicit solve for R > 1."""
    dims, R = (4, 5, 3), 3
    p, Y = _problem(5, dims, R, complex_)
    da, _, _ = brute.plain_step(p.y, p.init, 0.5)
    bad = cp.fast_step(Y, p.init, 0.5, w_form="printed")
    good = cp.fast_step(Y, p.init, 0.5)
    assert _rel(cp.flat(good.dA), cp.flat(da)) < 1e-10
    assert _rel(cp.flat(bad.dA), cp.flat(da)) > 1e-2


def test_transposed_F_is_caught(monkeypatch):
    """Planted mistake: reshaping f into F_n row-major instead of column-major."""
    dims, R = (4, 3, 5), 3
    p, Y = _problem(9, dims, R)
    da, _, _ = brute.plain_step(p.y, p.init, 0.3)
    orig = cp.unvec
    monkeypatch.setattr(cp, "unvec", lambda x, r, c: orig(x, r, c).T)
    bad = cp.fast_step(Y, p.init, 0.3)
    assert _rel(cp.flat(bad.dA), cp.flat(da)) > 1e-3


def test_wrong_K_index_is_caught(monkeypatch):
    """Planted mistake: K built without the commutation matrix."""
    dims, R = (4, 3, 5), 3
    p, Y = _problem(10, dims, R)
    da, _, _ = brute.plain_step(p.y, p.init, 0.3)
    monkeypatch.setattr(cp, "commutation", lambda R: np.eye(R * R))
    bad = cp.fast_step(Y, p.init, 0.3)
    assert _rel(cp.flat(bad.dA), cp.flat(da)) > 1e-3


@pytest.mark.parametrize("complex_", [False, True])
def test_hessian_low_rank_adjustment(complex_):
    """Theorem 4.2 (and Theorem 5.3): J^H J = G + Z K Z^H."""
    dims, R = (3, 4, 5, 3), 3
    p, _ = _problem(3, dims, R, complex_)
    A = p.init
    J = brute.jacobian(A)
    H = J.conj().T @ J
    C = cp.grams(A)
    Gam = cp.gammas(C)
    blocksG = [np.kron(Gam[n], np.eye(dims[n])) for n in range(len(A))]
    blocksZ = [np.kron(np.eye(R), A[n]) for n in range(len(A))]
    from scipy.linalg import block_diag
    G = block_diag(*blocksG)
    Z = block_diag(*blocksZ)
    K = cp.kernel_K(C)
    assert _rel(G + Z @ K @ Z.conj().T, H) < 1e-13


@pytest.mark.parametrize("N", [3, 4, 5])
def test_kernel_inverse_closed_form(N):
    """Theorem E.1: the printed blocks of K^-1 invert K."""
    rng = np.random.default_rng(N)
    R = 3
    A = [rng.standard_normal((5, R)) for _ in range(N)]
    C = cp.grams(A)
    K = cp.kernel_K(C)
    Ki = cp.kernel_K_inverse(C)
    assert np.abs(Ki @ K - np.eye(K.shape[0])).max() < 1e-10


@pytest.mark.parametrize("complex_", [False, True])
def test_euler_identity_of_jacobian(complex_):
    """Y_hat is homogeneous of degree N in a: J a = N vec(Y_hat)."""
    dims, R = (3, 4, 5), 2
    p, _ = _problem(2, dims, R, complex_)
    J = brute.jacobian(p.init)
    a = brute.param_vec(p.init)
    assert _rel(J @ a, len(dims) * brute.model_vec(p.init)) < 1e-13


@pytest.mark.parametrize("complex_", [False, True])
def test_matrix_free_products(complex_):
    dims, R = (4, 3, 5, 3), 3
    p, _ = _problem(4, dims, R, complex_)
    rng = np.random.default_rng(0)
    V = [rng.standard_normal(a.shape) + (1j * rng.standard_normal(a.shape) if complex_ else 0)
         for a in p.init]
    J = brute.jacobian(p.init)
    v = cp.flat(V)
    assert _rel(brute.jacobian_matvec(p.init, V), J @ v) < 1e-13
    assert _rel(cp.flat(brute.hessian_matvec(p.init, V)), J.conj().T @ (J @ v)) < 1e-13


@pytest.mark.parametrize("complex_", [False, True])
def test_zero_gradient_at_exact_rank_R(complex_):
    """Y = Y_hat(A) gives g = 0 and hence no update (Section 4.5, gradient)."""
    dims, R = (6, 5, 4), 3
    p, _ = _problem(6, dims, R, complex_)
    Y = cp.full(p.init)
    st = cp.fast_step(Y, p.init, 0.1)
    scale = np.linalg.norm(cp.flat(st.M))
    assert np.linalg.norm(cp.flat(st.g)) < 1e-13 * scale
    assert np.linalg.norm(cp.flat(st.dA)) < 1e-11 * np.linalg.norm(cp.flat(p.init))


def test_mu_to_infinity_is_steepest_descent():
    """mu da -> g with an O(||H|| / mu) remainder as mu grows."""
    dims, R = (5, 4, 3), 2
    p, Y = _problem(7, dims, R)
    errs = []
    for mu in (1e4, 1e6, 1e8):
        st = cp.fast_step(Y, p.init, mu)
        errs.append(_rel(mu * cp.flat(st.dA), cp.flat(st.g)))
    assert errs[0] > 50 * errs[1] and errs[1] > 50 * errs[2]
    assert errs[2] < 1e-5


@pytest.mark.parametrize("complex_", [False, True])
def test_mttkrp_brute_force_loop(complex_):
    """M_n[i_n, r] = sum over all entries y_i prod_{k != n} A_k[i_k, r] (conjugated factors for complex)."""
    dims, R = (3, 4, 2, 3), 2
    p, Y = _problem(8, dims, R, complex_)
    A = p.init
    for n in range(len(dims)):
        M = np.zeros((dims[n], R), dtype=Y.dtype)
        for idx in np.ndindex(*dims):
            for r in range(R):
                t = Y[idx]
                for k in range(len(dims)):
                    if k != n:
                        t = t * (A[k][idx[k], r].conj() if complex_ else A[k][idx[k], r])
                M[idx[n], r] += t
        assert _rel(cp.mttkrp(Y, A, n, conj=complex_), M) < 1e-13


@pytest.mark.parametrize("complex_", [False, True])
def test_full_model_equals_sum_of_outer_products(complex_):
    dims, R = (4, 3, 5, 2), 3
    p, _ = _problem(13, dims, R, complex_)
    assert _rel(cp.full(p.init).reshape(-1, order="F"), brute.model_vec(p.init)) < 1e-14


def test_mttkrp_mode1_is_plain_gemm_and_cross_mode_invariant():
    """Mode 1: the vec layout is Y_(1) column-major, so M_1 = reshape(y) @ KR.
    All modes: sum(A_n * M_n) = <Y, Y_hat> computed from the full model."""
    dims, R = (7, 5, 6, 4), 3
    p, Y = _problem(12, dims, R)
    A = p.init
    KR = np.ones((1, R))
    for a in A[1:]:
        KR = (a[:, None, :] * KR[None, :, :]).reshape(-1, R)
    M1 = p.y.reshape(dims[0], -1, order="F") @ KR
    assert _rel(cp.mttkrp(Y, A, 0), M1) < 1e-14
    inner = float(np.sum(Y * cp.full(A)))
    for n in range(len(dims)):
        assert abs(np.sum(A[n] * cp.mttkrp(Y, A, n)) - inner) < 1e-12 * abs(inner)


def _congruence(A, B):
    """Best column matching of factor sets A and B; product over modes of |cosines|."""
    from itertools import permutations
    R = A[0].shape[1]
    best = 0.0
    for perm in permutations(range(R)):
        score = 1.0
        for a, b in zip(A, B):
            for r in range(R):
                u, v = a[:, r], b[:, perm[r]]
                score = min(score, abs(np.vdot(u, v)) / (np.linalg.norm(u) * np.linalg.norm(v)))
        best = max(best, score)
    return best


@pytest.mark.parametrize("complex_", [False, True])
def test_noiseless_recovery(complex_):
    """Exact rank-R data from a perturbed truth: the fit reaches eps <= 1e-12
    and recovers the components up to order and scale."""
    dims, R = (8, 7, 6), 3
    p = cpgen.small_problem(21, dims, R, c=0.6, snr_db=None, complex_=complex_)
    Y = cp.as_tensor(p.y, dims)
    rng = np.random.default_rng(1)
    A0 = [a + 1e-2 * rng.standard_normal(a.shape) for a in p.truth]
    res = cp.fit(Y, A0, mu0=-1, tol=0.0, max_iters=60)
    assert res["eps"] <= 1e-12
    assert _congruence(res["A"], p.truth) > 1 - 1e-10


def test_fit_error_monotone_and_normalised():
    p = cpgen.cfg1()
    Y = cp.as_tensor(p.y, p.dims)
    res = cp.fit(Y, p.init, mu0=p.mu0, tol=0.0, max_iters=20, trace=True)
    errs = [h["err2"] for h in res["hist"]]
    assert all(b <= a for a, b in zip(errs, errs[1:]))
    norms = np.array([np.linalg.norm(a, axis=0) for a in res["A"]])
    assert np.allclose(norms, norms[0][None, :], rtol=1e-12)


def test_generator_gram_closed_form():
    rng = np.random.default_rng(0)
    for (I, R, c) in [(20, 3, 0.9), (50, 8, 0.95), (9, 9, 0.0)]:
        A = cpgen.collinear_factor(rng, I, R, c)
        target = (1 - c) * np.eye(R) + c * np.ones((R, R))
        assert np.abs(A.T @ A / I - target).max() < 1e-12


def test_generator_noise_level():
    rng = np.random.default_rng(0)
    y = rng.standard_normal(200000)
    yn, sigma = cpgen.add_noise(rng, y, 20.0)
    snr = 10 * np.log10(np.sum(y ** 2) / (sigma ** 2 * y.size))
    assert abs(snr - 20.0) < 1e-12
    assert abs(np.var(yn - y) / sigma ** 2 - 1) < 0.02


def test_generator_section6_angles_and_magnitudes():
    with open(os.path.join(GOLDEN, "section6_collinearity.json")) as fh:
        gold = json.load(fh)
    rng = np.random.default_rng(0)
    for nu, t1, tq in zip(gold["nu"], gold["theta_1r_deg"], gold["theta_qr_deg"]):
        A, _ = cpgen.nu_collinear_factors(rng, [12, 12, 12], 4, nu)
        a = A[0] / np.linalg.norm(A[0], axis=0)
        ang = np.degrees(np.arccos(np.clip(a.T @ a, -1, 1)))
        assert round(ang[0, 1]) == t1 and round(ang[0, 3]) == t1
        assert round(ang[1, 2]) == tq and round(ang[2, 3]) == tq
    A, _ = cpgen.nu_collinear_factors(rng, [12, 12, 12], 3, 2.0)
    a = A[0] / np.linalg.norm(A[0], axis=0)
    ang = np.degrees(np.arccos(a.T @ a))
    assert abs(ang[0, 1] - gold["nu2_theta_1r_deg_approx"]) < 1
    assert abs(ang[1, 2] - gold["nu2_theta_qr_deg_approx"]) < 1
    for nu, lam in gold["lambda_N3"].items():
        _, l = cpgen.nu_collinear_factors(rng, [5, 5, 5], 3, float(nu))
        assert abs(l[1] - lam) < 0.05


def test_generator_appendix_f_eigenvalues():
    """Appendix F: Y_(n) Y_(n)^T of the nu-collinear tensor has R-2 eigenvalues
    (x-1)(y-1), and lambda_1 + lambda_R, lambda_1 lambda_R as printed."""
    rng = np.random.default_rng(3)
    for (N, R, nu, I) in [(3, 5, 0.5, 20), (4, 4, 0.3, 8), (3, 6, 1.0, 15)]:
        A, _ = cpgen.nu_collinear_factors(rng, [I] * N, R, nu)
        Y = cp.as_tensor(cpgen.cp_tensor(A), [I] * N)
        ev = np.sort(np.linalg.eigvalsh(cp.unfold(Y, 0) @ cp.unfold(Y, 0).T))[::-1][:R]
        x = 1 + nu ** 2
        y = x ** (N - 1)
        assert np.allclose(ev[1:R - 1], (x - 1) * (y - 1), rtol=1e-9)
        assert abs(ev[0] + ev[-1] - (x * y + (R - 2) * (R + x + y) + 3)) < 1e-9 * ev[0]
        assert abs(ev[0] * ev[-1] - (x - 1) * (y - 1)) < 1e-9 * ev[0]
        # ||Y||^2 = trace(Sigma) = R^2 + (R-1)(xy - 1)  (the printed sigma^2 numerator
        # reads R^2 + (R-1)xy - 1, which only agrees for R = 2)
        assert abs(np.sum(Y ** 2) - (R ** 2 + (R - 1) * (x * y - 1))) < 1e-9 * np.sum(Y ** 2)


def test_phi_densities_section43():
    with open(os.path.join(GOLDEN, "section43_density.json")) as fh:
        gold = json.load(fh)
    dims, R = gold["dims"], gold["R"]
    N = len(dims)
    rng = np.random.default_rng(0)
    A = [rng.standard_normal((I, R)) for I in dims]
    C = cp.grams(A)
    Gt = [cp.damped_inverse(g, 0.1) for g in cp.gammas(C)]
    K = cp.kernel_K(C)
    Psi = cp.psi(Gt, C)
    Phi1 = np.eye(N * R * R) + Psi @ K
    Phi2 = cp.kernel_K_inverse(C) + Psi
    d1 = np.count_nonzero(np.abs(Phi1) > 1e-300) / Phi1.size
    d2 = np.count_nonzero(np.abs(Phi2) > 1e-300) / Phi2.size
    assert abs(d1 - ((N - 1) * R * R + 1) / (N * R * R)) < 1e-12
    assert abs(d2 - (R * R + N - 1) / (N * R * R)) < 1e-12


# ---- ALS warm-up (eq. ALS) -------------------------------------------------


def _brute_als_sweep(Y, A):
    """The ALS sweep as a plain least-squares problem per mode: the design
    matrix is built entry by entry from the definition of the Khatri-Rao
    product on the mode-n unfolding (first remaining index fastest), and each
    row of A^(n) comes from numpy's least-squares routine on it, with no Gram or
    Hadamard product involved."""
    A = [a.copy() for a in A]
    N = len(A)
    dims = Y.shape
    R = A[0].shape[1]
    dt = np.result_type(Y, *A)
    for n in range(N):
        others = [k for k in range(N) if k != n]
        cols = int(np.prod([dims[k] for k in others]))
        Z = np.zeros((cols, R), dtype=dt)
        Yn = np.zeros((dims[n], cols), dtype=dt)
        for j, idx in enumerate(np.ndindex(*[dims[k] for k in reversed(others)])):
            idx = idx[::-1]  # first remaining index fastest
            for r in range(R):
                Z[j, r] = np.prod([A[k][i, r] for k, i in zip(others, idx)])
            full_idx = [0] * N
            for k, i in zip(others, idx):
                full_idx[k] = i
            for i_n in range(dims[n]):
                full_idx[n] = i_n
                Yn[i_n, j] = Y[tuple(full_idx)]
        A[n] = np.linalg.lstsq(Z, Yn.T, rcond=None)[0].T
    return A


@pytest.mark.parametrize("dims,R,cplx", [((4, 3, 5), 2, False), ((5, 4, 3), 3, False), ((3, 4, 3, 4), 2, False),
                                          ((4, 3, 5), 2, True), ((3, 4, 3, 4), 3, True)])
def test_als_sweep_matches_brute_force_least_squares(dims, R, cplx):
    rng = np.random.default_rng(11 + R)

    def draw(shape):
        x = rng.standard_normal(shape)
        return x + 1j * rng.standard_normal(shape) if cplx else x
    Y = draw(dims)
    A0 = [draw((I, R)) for I in dims]
    got = cp.als_sweep(Y, A0)
    want = _brute_als_sweep(Y, A0)
    for g, w in zip(got, want):
        assert _rel(g, w) < 1e-10


def test_als_sweep_fixed_point_at_exact_factors():
    # an exact rank-R tensor built from A is reproduced exactly, so every mode's
    # least-squares update returns the same factor
    rng = np.random.default_rng(5)
    for dims, R in SHAPES:
        A = [rng.standard_normal((I, R)) for I in dims]
        Y = cp.full(A)
        A1 = cp.als_sweep(Y, A)
        for a, b in zip(A1, A):
            assert _rel(a, b) < 1e-9


def test_als_last_mode_solves_its_normal_equations_and_error_decreases():
    rng = np.random.default_rng(9)
    dims, R = (6, 5, 7), 3
    truth = [rng.standard_normal((I, R)) for I in dims]
    Y = cp.full(truth) + 0.05 * rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    prev = cp.residual_norm2(Y, A)
    for _ in range(4):
        A = cp.als_sweep(Y, A)
        # the gradient with respect to the last updated factor vanishes:
        # Y_(N) KR - A^(N) KR^T KR = 0 with KR^T KR from the unfolding itself
        N = len(A)
        KR = cp.kr_except(A, N - 1)
        resid = cp.unfold(Y, N - 1) @ KR - A[N - 1] @ (KR.T @ KR)
        assert np.linalg.norm(resid) < 1e-10 * np.linalg.norm(cp.unfold(Y, N - 1) @ KR)
        err = cp.residual_norm2(Y, A)
        assert err <= prev * (1 + 1e-12)
        prev = err


def test_als_planted_all_mode_gamma_fails_the_pin():
    # the Hadamard over all modes (Gamma of Theorem 4.1's simplified form) in
    # place of Gamma^(n) breaks the least-squares update
    rng = np.random.default_rng(12)
    dims, R = (4, 3, 5), 2
    Y = rng.standard_normal(dims)
    A = [rng.standard_normal((I, R)) for I in dims]
    B = [a.copy() for a in A]
    for n in range(3):
        M = cp.mttkrp(Y, B, n)
        G = cp.hadamard_except(cp.grams(B), set())
        B[n] = np.linalg.solve(G, M.T).T
    want = _brute_als_sweep(Y, A)
    assert max(_rel(b, w) for b, w in zip(B, want)) > 1e-3


# ---- SVD initialisation (Section 4.5) ----------------------------------------


def test_svd_init_matches_eigenvectors_of_the_mode_gram():
    # a different route: eigenvectors of Y_(n) Y_(n)^T built by an explicit
    # loop over the mode-n fibres, from a symmetric eigensolver
    rng = np.random.default_rng(21)
    dims, R = (7, 6, 5), 3
    Y = rng.standard_normal(dims)
    A, S = cp.svd_init(Y, R)
    for n in range(3):
        G = np.zeros((dims[n], dims[n]))
        others = [k for k in range(3) if k != n]
        for idx in np.ndindex(*[dims[k] for k in others]):
            sl = [slice(None)] * 3
            for k, i in zip(others, idx):
                sl[k] = i
            f = Y[tuple(sl)]
            G += np.outer(f, f)
        w, V = np.linalg.eigh(G)
        V = cp.canonical_signs(V[:, ::-1][:, :R])
        assert np.allclose(S[n] ** 2, w[::-1][:R], rtol=1e-10)
        assert np.linalg.norm(A[n] - V) < 1e-9
        assert np.linalg.norm(A[n].T @ A[n] - np.eye(R)) < 1e-12


def test_svd_init_spans_the_factors_of_an_exact_rank_r_tensor():
    rng = np.random.default_rng(22)
    dims, R = (8, 7, 9), 3
    F = [rng.standard_normal((I, R)) for I in dims]
    A, _ = cp.svd_init(cp.full(F), R)
    for a, f in zip(A, F):
        # the projector onto span(A^(n)) reproduces the true factor
        assert np.linalg.norm(a @ (a.T @ f) - f) < 1e-10 * np.linalg.norm(f)


def test_svd_init_complex_matches_hermitian_gram_eigenvectors():
    # complex tensors (Section 5): the left singular vectors of Y_(n) are the
    # eigenvectors of the Hermitian Y_(n) Y_(n)^H, built here by a fibre loop
    rng = np.random.default_rng(23)
    dims, R = (6, 5, 7), 3
    Y = rng.standard_normal(dims) + 1j * rng.standard_normal(dims)
    A, S = cp.svd_init(Y, R)
    for n in range(3):
        G = np.zeros((dims[n], dims[n]), dtype=complex)
        others = [k for k in range(3) if k != n]
        for idx in np.ndindex(*[dims[k] for k in others]):
            sl = [slice(None)] * 3
            for k, i in zip(others, idx):
                sl[k] = i
            f = Y[tuple(sl)]
            G += np.outer(f, np.conj(f))
        w, V = np.linalg.eigh(G)
        V = cp.canonical_signs(V[:, ::-1][:, :R])
        assert np.allclose(S[n] ** 2, w[::-1][:R], rtol=1e-10)
        assert np.linalg.norm(A[n] - V) < 1e-9
        assert np.linalg.norm(A[n].conj().T @ A[n] - np.eye(R)) < 1e-12
        for r in range(R):  # the canonical phase: largest entry real and positive
            k = int(np.argmax(np.abs(A[n][:, r])))
            assert abs(A[n][k, r].imag) < 1e-15 and A[n][k, r].real > 0


# ---- gain ratio, mu0 and the normalisations (Section 4.5, eq. mu0, Section 2) ----


def _linear_model_decrease(y_vec, A, dA):
    """||e||^2 - ||e - J da||^2 with J formed explicitly: the decrease that the
    linearised model predicts for the step da (e = y - y_hat)."""
    J = brute.jacobian(A)
    e = y_vec - brute.model_vec(A)
    r = e - J @ brute.param_vec(dA)
    return float(np.sum(np.abs(e) ** 2) - np.sum(np.abs(r) ** 2))


@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("mu", [1e-2, 1.0, 30.0])
def test_gain_denominator_is_the_linear_model_decrease(mu, complex_):
    """The denominator of rho (Section 4.5) is the decrease of the linearised
    residual: for da = (J^H J + mu I)^-1 J^H e,
    ||e||^2 - ||e - J da||^2 = 2 Re(da^H g) - da^H H da = Re(da^H (g + mu da)).
    The left side is computed from the explicit Jacobian only."""
    dims, R = (4, 3, 5), 3
    p, Y = _problem(31, dims, R, complex_)
    st = cp.fast_step(Y, p.init, mu)
    ref = _linear_model_decrease(p.y, p.init, st.dA)
    got = cp.gain_denominator(st.dA, st.g, mu)
    assert ref > 0
    assert abs(got - ref) <= 1e-10 * ref


def test_gain_denominator_planted_mistakes_fail():
    """A sign slip on the mu term, or the mu term dropped, misses the linear-model decrease."""
    dims, R, mu = (4, 3, 5), 3, 1.0
    p, Y = _problem(32, dims, R)
    st = cp.fast_step(Y, p.init, mu)
    ref = _linear_model_decrease(p.y, p.init, st.dA)
    assert abs(cp.gain_denominator(st.dA, st.g, -mu) - ref) > 1e-3 * ref
    assert abs(cp.gain_denominator(st.dA, st.g, 0.0) - ref) > 1e-3 * ref


@pytest.mark.parametrize("complex_", [False, True])
def test_mu0_is_tau_times_max_diag_of_explicit_hessian(complex_):
    """eq. mu0, first form: mu0 = tau max diag(J^H J), J formed explicitly."""
    dims, R, tau = (4, 5, 3, 3), 3, 1e-3
    p, _ = _problem(33, dims, R, complex_)
    A = [a * s for a, s in zip(p.init, (0.5, 2.0, 3.0, 0.7))]   # modes of unequal scale
    J = brute.jacobian(A)
    ref = tau * float(np.max(np.real(np.sum(np.abs(J) ** 2, axis=0))))
    assert abs(cp.mu0_from_tau(A, tau) - ref) <= 1e-13 * ref


def test_mu0_last_form_holds_for_unit_modes():
    """eq. mu0, last form: with unit-norm columns in modes 1..N-1 the rule is
    tau max{1, diag C^(N)}."""
    dims, R, tau = (5, 4, 6), 3, 1e-2
    p, _ = _problem(34, dims, R)
    A = cp.normalize_unit_except_last([a * 3.0 for a in p.init])
    ref = tau * max(1.0, float(np.max(np.diag(A[-1].T @ A[-1]))))
    assert abs(cp.mu0_from_tau(A, tau) - ref) <= 1e-13 * ref


def test_mu0_planted_gram_instead_of_gamma_fails(monkeypatch):
    """Planted mistake: the maximum over diag C^(n) instead of diag Gamma^(n)."""
    dims, R, tau = (4, 5, 3), 3, 1e-3
    p, _ = _problem(35, dims, R)
    A = [a * s for a, s in zip(p.init, (0.5, 2.0, 3.0))]
    ref = tau * float(np.max(np.sum(brute.jacobian(A) ** 2, axis=0)))
    monkeypatch.setattr(cp, "gammas", lambda C: C)
    assert abs(cp.mu0_from_tau(A, tau) - ref) > 1e-3 * ref


@pytest.mark.parametrize("complex_", [False, True])
def test_normalize_unit_except_last(complex_):
    """Section 2 convention: Y_hat unchanged, unit columns in modes 1..N-1 and
    the last mode's column norms equal to prod_n ||a^(n)_r||."""
    dims, R = (4, 3, 5, 3), 3
    p, _ = _problem(36, dims, R, complex_)
    A = [a * s for a, s in zip(p.init, (0.5, 2.0, 3.0, 0.7))]
    out = cp.normalize_unit_except_last(A)
    assert _rel(brute.model_vec(out), brute.model_vec(A)) < 1e-14
    for n in range(len(dims) - 1):
        assert np.allclose(np.linalg.norm(out[n], axis=0), 1.0, rtol=1e-14, atol=0)
    lam = np.prod([np.linalg.norm(a, axis=0) for a in A], axis=0)
    assert np.allclose(np.linalg.norm(out[-1], axis=0), lam, rtol=1e-13, atol=0)


def test_normalize_balanced_keeps_the_model():
    """Algorithm 1 normalisation: Y_hat unchanged and every mode's column norm
    equal to lambda_r^(1/N)."""
    dims, R = (4, 3, 5), 3
    p, _ = _problem(37, dims, R)
    A = [a * s for a, s in zip(p.init, (0.5, 2.0, 3.0))]
    out = cp.normalize_balanced(A)
    assert _rel(brute.model_vec(out), brute.model_vec(A)) < 1e-14
    lam = np.prod([np.linalg.norm(a, axis=0) for a in A], axis=0)
    for a in out:
        assert np.allclose(np.linalg.norm(a, axis=0), lam ** (1 / 3), rtol=1e-14, atol=0)


def test_normalize_planted_missing_last_mode_scale_fails(monkeypatch):
    """Planted mistake: modes 1..N-1 scaled to unit norm without moving the
    magnitude into mode N changes the model."""
    dims, R = (4, 3, 5), 3
    p, _ = _problem(38, dims, R)
    A = [a * s for a, s in zip(p.init, (0.5, 2.0, 3.0))]

    def bad(A):
        out = [a.copy() for a in A]
        for n in range(len(A) - 1):
            out[n] = out[n] / np.linalg.norm(out[n], axis=0)
        return out

    assert _rel(brute.model_vec(bad(A)), brute.model_vec(A)) > 1e-2


# ---- damping rules on a run of rejected trials (Section 4.5) ------------------


def _null_step_fit(mu_rule):
    """At mu0 = 1e25 every step is far below half an ulp of the factors, so
    A + da == A, the residual is unchanged and every trial is rejected."""
    dims, R = (5, 4, 3), 2
    p, Y = _problem(39, dims, R)
    return cp.fit(Y, p.init, mu0=1e25, tol=0.0, max_iters=100, trace=True, mu_rule=mu_rule)


def test_paper_rule_doubles_mu_per_rejection():
    """Section 4.5 as printed: after k rejections mu = mu0 2^k; the first mu
    above 1e30 stops the fit, here after k = 17 (2^17 > 1e5 > 2^16)."""
    res = _null_step_fit("paper")
    assert res["reason"] == cp.STOP_MU and res["accepted"] == 0
    assert res["iters"] == 17
    mus = [h["mu"] for h in res["hist"]]
    assert mus == [1e25 * 2.0 ** k for k in range(17)]


def test_nielsen_rule_closed_form_on_rejection_runs():
    """Nielsen's rule: with nu = 2 after an acceptance (or at the start), j
    consecutive rejections multiply mu by 2 * 4 * ... * 2^j = 2^(j(j+1)/2).
    From 1e25 the fit passes 1e30 after j = 6 (2^21 > 1e5 > 2^15)."""
    res = _null_step_fit("nielsen")
    assert res["reason"] == cp.STOP_MU and res["accepted"] == 0
    assert res["iters"] == 6
    mus = [h["mu"] for h in res["hist"]]
    assert mus == [1e25 * 2.0 ** (j * (j + 1) // 2) for j in range(6)]
    assert res["mu"] == 1e25 * 2.0 ** 21


def test_nielsen_rule_resets_nu_on_acceptance():
    """On a real fit the two rules agree up to the first rejection; after an
    acceptance the next rejection multiplies mu by 2 again."""
    p = cpgen.cfg1()
    Y = cp.as_tensor(p.y, p.dims)
    a = cp.fit(Y, p.init, mu0=1e-3, tol=0.0, max_iters=30, trace=True, mu_rule="paper")["hist"]
    b = cp.fit(Y, p.init, mu0=1e-3, tol=0.0, max_iters=30, trace=True, mu_rule="nielsen")["hist"]
    first_rej = next(i for i, h in enumerate(a) if not h["accepted"])
    for i in range(first_rej + 1):
        assert a[i]["mu"] == b[i]["mu"]
    run = 0
    for h0, h1 in zip(b, b[1:]):
        run = 0 if h0["accepted"] else run + 1
        if not h0["accepted"]:
            assert h1["mu"] == h0["mu"] * 2.0 ** run

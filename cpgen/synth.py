"""Synthetic CP problems (Section 6 of the paper and the stated workloads).

All draws use NumPy's PCG64 (`numpy.random.default_rng(seed)`) in float64.
Tensors are returned as 1-D float64 (or complex128) arrays holding vec(Y)
with the first index fastest (column-major), which is the paper's
vectorisation (Section 2, Kolda's convention).  Factors are float64
(complex128) arrays of shape (I_n, R) in Fortran order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _gram_target_chol(R: int, c: float) -> np.ndarray:
    """Lower Cholesky factor of (1-c) I + c 11^T (pairwise correlation c)."""
    S = (1.0 - c) * np.eye(R) + c * np.ones((R, R))
    return np.linalg.cholesky(S)


def collinear_factor(rng: np.random.Generator, I: int, R: int, c: float,
                     complex_: bool = False) -> np.ndarray:
    """I x R factor whose columns have pairwise correlation c.

    A = sqrt(I) * Q L^T with Q an orthonormal basis of a Gaussian I x R draw
    and L L^T = (1-c) I + c 11^T, so that A^T A / I = (1-c) I + c 11^T holds
    exactly (up to rounding).  When I < R no orthonormal Q exists; a Gaussian
    G replaces Q and the identity then holds only in expectation.
    """
    L = _gram_target_chol(R, c)
    if complex_:
        G = (rng.standard_normal((I, R)) + 1j * rng.standard_normal((I, R))) / np.sqrt(2.0)
    else:
        G = rng.standard_normal((I, R))
    if I >= R:
        Q, _ = np.linalg.qr(G)
        A = np.sqrt(I) * (Q @ L.T)
    else:
        A = G @ L.T
    return np.asfortranarray(A)


def nu_collinear_factors(rng: np.random.Generator, dims, R: int, nu: float):
    """The paper's collinear generator (Section 6): a_r = u_1 + nu u_r for r > 1.

    U is a random orthonormal I_n x R matrix; a_1 = u_1.  Returned with the
    magnitudes lambda_1 = 1, lambda_r = (1 + nu^2)^(N/2) of that section.
    """
    N = len(dims)
    out = []
    for I in dims:
        U, _ = np.linalg.qr(rng.standard_normal((I, R)))
        A = U.copy()
        A[:, 1:] = U[:, [0]] + nu * U[:, 1:]
        out.append(np.asfortranarray(A))
    lam = np.ones(R)
    lam[1:] = (1.0 + nu * nu) ** (N / 2.0)
    return out, lam


def cp_tensor(factors, lam=None) -> np.ndarray:
    """vec of sum_r lam_r a^(1)_r o ... o a^(N)_r, first index fastest.

    Built as A^(1) times the transposed Khatri-Rao product of the remaining
    factors, which is the mode-1 unfolding of the CP model.
    """
    R = factors[0].shape[1]
    if lam is None:
        lam = np.ones(R)
    kr = np.ones((1, R), dtype=np.result_type(*factors))
    for A in factors[1:]:
        # rows of kr are indexed with the earlier modes fastest
        kr = (A[:, None, :] * kr[None, :, :]).reshape(-1, R)
    Y1 = (factors[0] * lam[None, :]) @ kr.T
    return np.asarray(Y1, order="F").reshape(-1, order="F")


def add_noise(rng: np.random.Generator, y: np.ndarray, snr_db: float) -> tuple[np.ndarray, float]:
    """Additive white Gaussian noise at SNR = 10 log10(||Y||^2 / (sigma^2 J)).

    The sign of the printed SNR formula in Section 6 is read as the usual
    positive one (the commented formula for sigma beside it agrees).
    """
    J = y.size
    sigma = 10.0 ** (-snr_db / 20.0) * np.linalg.norm(y) / np.sqrt(J)
    if np.iscomplexobj(y):
        n = (rng.standard_normal(J) + 1j * rng.standard_normal(J)) / np.sqrt(2.0)
    else:
        n = rng.standard_normal(J)
    return y + sigma * n, sigma


def random_init(rng: np.random.Generator, dims, R: int, complex_: bool = False):
    """Independent N(0,1) factors (random initialisation, Algorithm 1)."""
    out = []
    for I in dims:
        if complex_:
            A = (rng.standard_normal((I, R)) + 1j * rng.standard_normal((I, R))) / np.sqrt(2.0)
        else:
            A = rng.standard_normal((I, R))
        out.append(np.asfortranarray(A))
    return out


@dataclass
class Problem:
    dims: tuple
    R: int
    y: np.ndarray                    # vec(Y), first index fastest, float64/complex128
    truth: list                      # factors of the noiseless model (lambda folded into the last)
    init: list                       # starting factors
    mu0: float = -1.0                # <= 0 means "derive from tau" (paper's mu0 rule)
    max_iters: int = 50
    tol: float = 0.0
    sigma: float = 0.0
    meta: dict = field(default_factory=dict)


def small_problem(seed: int, dims, R: int, c: float = 0.5, snr_db: float | None = 30.0,
                  complex_: bool = False) -> Problem:
    """Generic small seeded problem used by tests (collinearity c in every mode)."""
    rng = np.random.default_rng(seed)
    truth = [collinear_factor(rng, I, R, c, complex_) for I in dims]
    y = cp_tensor(truth)
    sigma = 0.0
    if snr_db is not None:
        y, sigma = add_noise(rng, y, snr_db)
    init = random_init(rng, dims, R, complex_)
    return Problem(tuple(dims), R, y, truth, init, sigma=sigma)


def cfg1(seed: int = 1) -> Problem:
    """3-way 20x20x20, R=3, mode-1 columns at correlation 0.9, 30 dB, mu0=1, 50 trials."""
    rng = np.random.default_rng(seed)
    dims, R = (20, 20, 20), 3
    truth = [collinear_factor(rng, dims[0], R, 0.9)]
    truth += [np.asfortranarray(rng.standard_normal((I, R))) for I in dims[1:]]
    y = cp_tensor(truth)
    y, sigma = add_noise(rng, y, 30.0)
    init = random_init(rng, dims, R)
    return Problem(dims, R, y, truth, init, mu0=1.0, max_iters=50, tol=0.0, sigma=sigma,
                   meta={"name": "cfg1", "c": 0.9, "snr_db": 30.0})


def cfg2(seed: int = 2, dims=(100, 100, 100, 100)) -> Problem:
    """4-way 100^4, R=10, correlation 0.95 in all modes, lambda_r = 10^U(0,2), 20 dB."""
    rng = np.random.default_rng(seed)
    R = 10
    truth = [collinear_factor(rng, I, R, 0.95) for I in dims]
    lam = 10.0 ** rng.uniform(0.0, 2.0, size=R)
    truth[-1] = np.asfortranarray(truth[-1] * lam[None, :])
    y = cp_tensor(truth)
    y, sigma = add_noise(rng, y, 20.0)
    init = random_init(rng, dims, R)
    return Problem(tuple(dims), R, y, truth, init, mu0=-1.0, max_iters=20, tol=0.0, sigma=sigma,
                   meta={"name": "cfg2", "c": 0.95, "snr_db": 20.0, "lam": lam})


def cfg3(seed: int = 3, dims=(500, 500, 500), R: int = 30) -> Problem:
    """3-way 500^3, R=30, lambda_r = 10^(3(r-1)/(R-1)), correlation 0.9 in mode 3, 25 dB
    (smaller dims and R give samples of the same recipe)."""
    rng = np.random.default_rng(seed)
    truth = [np.asfortranarray(rng.standard_normal((I, R))) for I in dims[:-1]]
    truth.append(collinear_factor(rng, dims[-1], R, 0.9))
    lam = 10.0 ** (3.0 * np.arange(R) / (R - 1))
    truth[-1] = np.asfortranarray(truth[-1] * lam[None, :])
    y = cp_tensor(truth)
    y, sigma = add_noise(rng, y, 25.0)
    init = random_init(rng, dims, R)
    return Problem(tuple(dims), R, y, truth, init, mu0=-1.0, max_iters=20, tol=0.0, sigma=sigma,
                   meta={"name": "cfg3", "c": 0.9, "snr_db": 25.0, "lam": lam})


def cfg4(seed: int = 4, count: int = 1024, max_iters: int = 200, tol: float = 1e-8):
    """Many small uneven 3-way fits: I_n ~ U{8..64}, R ~ U{2..8}, c ~ U[0,0.95], SNR ~ U[20,40]."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        dims = tuple(int(v) for v in rng.integers(8, 65, size=3))
        R = int(rng.integers(2, 9))
        c = float(rng.uniform(0.0, 0.95))
        snr = float(rng.uniform(20.0, 40.0))
        truth = [collinear_factor(rng, I, R, c) for I in dims]
        y = cp_tensor(truth)
        y, sigma = add_noise(rng, y, snr)
        init = random_init(rng, dims, R)
        out.append(Problem(dims, R, y, truth, init, mu0=-1.0, max_iters=max_iters, tol=tol,
                           sigma=sigma, meta={"name": "cfg4", "index": b, "c": c, "snr_db": snr}))
    return out


def svd_start_block(rng: np.random.Generator, dims, block: int) -> np.ndarray:
    """Random start blocks of the SVD initialisation: N(0,1) entries, mode n's
    I_n x block column-major block after those of the earlier modes."""
    return np.concatenate([rng.standard_normal((block, int(I))).reshape(-1) for I in dims])


def svd_start_block_complex(rng: np.random.Generator, dims, block: int) -> np.ndarray:
    """Complex start blocks: real and imaginary parts N(0,1), same layout."""
    re = svd_start_block(rng, dims, block)
    return re + 1j * svd_start_block(rng, dims, block)

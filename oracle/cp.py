"""Plain FP64 implementation of the fast damped Gauss-Newton step for CP.

Follows the paper (Phan, Tichavsky, Cichocki, "Low complexity damped
Gauss-Newton algorithms for CANDECOMP/PARAFAC") step by step:

* Section 2 / Notation 2.1: unfoldings Y_(n) and Khatri-Rao products with the
  first mode fastest.
* Section 3, eq. (ALS): C^(n) = A^(n)T A^(n), Gamma^(n) = Hadamard of C^(k), k != n.
* Theorem 4.1 (fast dGN): Gamma^(n,m), K, Gamma~_mu, A_mu, Psi_mu, w_mu and
  the boxed factor update.
* Lemma 4.4 / Appendix D: the Jacobian-free products.  The simplified w_mu
  printed in Theorem 4.1 (with the all-mode Hadamard Gamma) disagrees with the
  unsimplified line of Appendix D; the oracle uses the unsimplified form
  w_n = vec(A^(n)T (A^(n)_mu - A^(n) Gamma^(n) Gamma~^(n))), which is what the
  explicit solve confirms (tests/test_oracle_pins.py plants the printed form
  and shows it fails).
* Section 4.3: fLMa, f = K (I + Psi K)^-1 w, and fLMb, f = (K^-1 + Psi)^-1 w
  with K^-1 from Theorem E.1.
* Section 4.5: the gain ratio, acceptance and the damping update.
* Section 5: the complex variant.  Where Section 5 writes Gamma~ without a
  transpose inside A_mu and the update, the oracle uses (Gamma^(n)T + mu I)^-1,
  which is what G~_mu = blkdiag((Gamma^(n) + mu I)^-1 (x) I) gives when applied
  to vec of an I_n x R matrix; Psi keeps (Gamma^(n) + mu I)^-1.

Everything is float64 / complex128 NumPy.  Library routines (matmul, solve,
cholesky) serve as single steps; nothing is blocked, fused or reordered.
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------
# Multilinear algebra (Section 2)
# ----------------------------------------------------------------------------


def as_tensor(y: np.ndarray, dims) -> np.ndarray:
    """vec(Y) (first index fastest) -> N-way array."""
    return np.asarray(y).reshape(tuple(dims), order="F")


def unfold(Y: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding Y_(n): I_n x prod_{k!=n} I_k, remaining indices in
    increasing mode order with the earliest fastest (Kolda's convention)."""
    return np.moveaxis(Y, n, 0).reshape(Y.shape[n], -1, order="F")


def khatri_rao(mats) -> np.ndarray:
    """Column-wise Kronecker product B1 (.) B2 (.) ... ; the last factor's row
    index varies fastest, so khatri_rao([A_N, ..., A_1]) has i_1 fastest."""
    R = mats[0].shape[1]
    out = mats[0]
    for B in mats[1:]:
        out = np.einsum("ir,jr->ijr", out, B).reshape(-1, R)
    return out


def kr_except(A, n: int) -> np.ndarray:
    """The Khatri-Rao product A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1)."""
    return khatri_rao([A[k] for k in reversed(range(len(A))) if k != n])


def mttkrp(Y: np.ndarray, A, n: int, conj: bool = False) -> np.ndarray:
    """Y_(n) (Khatri-Rao of A^(k), k != n); with conj the factors are conjugated
    (Theorem 5.4, complex gradient)."""
    KR = kr_except(A, n)
    if conj:
        KR = KR.conj()
    return unfold(Y, n) @ KR


def full(A) -> np.ndarray:
    """The CP model (eq. CP) through its mode-1 unfolding (Section 2):
    Y_hat_(1) = A^(1) (A^(N) (.) ... (.) A^(2))^T, folded back to N-way."""
    dims = [a.shape[0] for a in A]
    Y1 = A[0] @ kr_except(A, 0).T
    return Y1.reshape(dims, order="F")


def residual_norm2(Y: np.ndarray, A) -> float:
    """||Y - Y_hat||_F^2 by direct summation of the residual."""
    E = Y - full(A)
    return float(np.sum(np.abs(E) ** 2))


# ----------------------------------------------------------------------------
# Gram and Hadamard products (eq. ALS, Theorem 4.1)
# ----------------------------------------------------------------------------


def grams(A):
    """C^(n) = A^(n)H A^(n)  (A^(n)T A^(n) for real factors)."""
    return [a.conj().T @ a for a in A]


def hadamard_except(C, skip) -> np.ndarray:
    """Hadamard product of C^(k) over k not in `skip`."""
    R = C[0].shape[0]
    out = np.ones((R, R), dtype=np.result_type(*C))
    for k, c in enumerate(C):
        if k not in skip:
            out = out * c
    return out


def gammas(C):
    """Gamma^(n) = Hadamard_{k != n} C^(k)."""
    return [hadamard_except(C, {n}) for n in range(len(C))]


def damped_inverse(G: np.ndarray, mu: float) -> np.ndarray:
    """(G + mu I)^-1 for Hermitian positive definite G + mu I, via Cholesky."""
    R = G.shape[0]
    L = np.linalg.cholesky(G + mu * np.eye(R))
    Linv = np.linalg.solve(L, np.eye(R))
    return Linv.conj().T @ Linv


# ----------------------------------------------------------------------------
# Kernel matrix K (eq. Knm_a) and its inverse (Theorem E.1)
# ----------------------------------------------------------------------------


def commutation(R: int) -> np.ndarray:
    """P_R with P_R vec(X^T) = vec(X) for R x R X."""
    P = np.zeros((R * R, R * R))
    for i in range(R):
        for j in range(R):
            # vec(X)[i + jR] = X[i, j] = X^T[j, i] = vec(X^T)[j + iR]
            P[i + j * R, j + i * R] = 1.0
    return P


def vec(X: np.ndarray) -> np.ndarray:
    return np.asarray(X).reshape(-1, order="F")


def unvec(x: np.ndarray, rows: int, cols: int) -> np.ndarray:
    return np.asarray(x).reshape(rows, cols, order="F")


def kernel_K(C) -> np.ndarray:
    """K = [ (1 - delta_nm) P_R diag(vec Gamma^(n,m)) ]_{n,m}, NR^2 x NR^2."""
    N = len(C)
    R = C[0].shape[0]
    R2 = R * R
    P = commutation(R)
    K = np.zeros((N * R2, N * R2), dtype=np.result_type(*C))
    for n in range(N):
        for m in range(N):
            if n == m:
                continue
            Gnm = hadamard_except(C, {n, m})
            K[n * R2:(n + 1) * R2, m * R2:(m + 1) * R2] = P @ np.diag(vec(Gnm))
    return K


def kernel_K_inverse(C) -> np.ndarray:
    """Theorem E.1: blocks (1/(N-1) - delta_nm) diag(vec(C^(n) * C^(m) / Gamma)) P_R,
    with Gamma the Hadamard product of all C^(k).  Needs every Gamma entry != 0."""
    N = len(C)
    R = C[0].shape[0]
    R2 = R * R
    P = commutation(R)
    Gall = hadamard_except(C, set())
    Ki = np.zeros((N * R2, N * R2), dtype=np.result_type(*C))
    for n in range(N):
        for m in range(N):
            coef = 1.0 / (N - 1) - (1.0 if n == m else 0.0)
            D = np.diag(vec(C[n] * C[m] / Gall))
            Ki[n * R2:(n + 1) * R2, m * R2:(m + 1) * R2] = coef * (D @ P)
    return Ki


def psi(Gt, C) -> np.ndarray:
    """Psi_mu = blkdiag(Gamma~^(n) (x) C^(n))  (eq. ZiGZ_LM_a)."""
    N = len(C)
    R = C[0].shape[0]
    R2 = R * R
    out = np.zeros((N * R2, N * R2), dtype=np.result_type(*Gt, *C))
    for n in range(N):
        out[n * R2:(n + 1) * R2, n * R2:(n + 1) * R2] = np.kron(Gt[n], C[n])
    return out


# ----------------------------------------------------------------------------
# The fast step (Theorem 4.1, Lemma 4.4, Section 4.3; Section 5 for complex)
# ----------------------------------------------------------------------------


class Step(dict):
    """Attribute access to the quantities of one fast step."""

    __getattr__ = dict.__getitem__


def fast_step(Y: np.ndarray, A, mu: float, variant: str = "a", w_form: str = "appendix") -> Step:
    """One trial step at damping mu.  Returns the new factors and the pieces.

    Y is the N-way array, A a list of I_n x R factors.  `variant` 'a' solves
    with Phi_1 = I + Psi K (fLMa), 'b' with Phi_2 = K^-1 + Psi (fLMb).
    `w_form` 'appendix' is the unsimplified w of Appendix D (the oracle's
    reading); 'printed' is the simplified form printed in Theorem 4.1 and is
    only used by a test that shows it is wrong.
    """
    N = len(A)
    R = A[0].shape[1]
    R2 = R * R
    cplx = any(np.iscomplexobj(a) for a in A) or np.iscomplexobj(Y)
    I_R = np.eye(R)

    C = grams(A)                                           # C^(n)
    Gam = gammas(C)                                        # Gamma^(n)
    # Gamma~^(n) = (Gamma^(n) + mu I)^-1 enters Psi; the factor-side inverse is
    # transposed in the complex case (Section 5, see module docstring).
    Gt_psi = [damped_inverse(Gam[n], mu) for n in range(N)]
    Gt_fac = [g.T if cplx else g for g in Gt_psi]
    Gam_fac = [g.T if cplx else g for g in Gam]            # Gamma^(n)T in Section 5

    M = [mttkrp(Y, A, n, conj=cplx) for n in range(N)]     # Y_(n) (KR of A^(k)[*])
    A_mu = [M[n] @ Gt_fac[n] for n in range(N)]            # damped ALS factor
    G = [M[n] - A[n] @ Gam_fac[n] for n in range(N)]       # gradient blocks (Sec. 4.5 / Thm 5.4)
    P = [A_mu[n] - A[n] @ Gam_fac[n] @ Gt_fac[n] for n in range(N)]   # G~_mu g (Lemma 4.4)

    if w_form == "appendix":
        w = np.concatenate([vec(A[n].conj().T @ P[n]) for n in range(N)])
    elif w_form == "printed":
        Gall = hadamard_except(C, set())
        w = np.concatenate([vec(A[n].conj().T @ A_mu[n] - Gall @ Gt_fac[n]) for n in range(N)])
    else:
        raise ValueError(w_form)

    K = kernel_K(C)
    Psi = psi(Gt_psi, C)
    if variant == "a":
        Phi = np.eye(N * R2) + Psi @ K                     # Phi_1 (fLMa)
        f = K @ np.linalg.solve(Phi, w)
    elif variant == "b":
        Phi = kernel_K_inverse(C) + Psi                    # Phi_2 (fLMb)
        f = np.linalg.solve(Phi, w)
    else:
        raise ValueError(variant)

    F = [unvec(f[n * R2:(n + 1) * R2], R, R) for n in range(N)]   # frontal slices of F
    # boxed update (equ_fast_low_LM1a): A_mu + A (I - (F_n + Gamma) Gamma~)
    A_new = [A_mu[n] + A[n] @ (I_R - (F[n] + Gam_fac[n]) @ Gt_fac[n]) for n in range(N)]
    # the step da = H_mu^-1 g itself (Section 4.5 defines rho with it): the boxed
    # update minus A, i.e. P_n - A_n F_n Gamma~_n; formed directly rather than as
    # A_new - A, which cancels to zero once da is below the factors' rounding
    dA = [P[n] - A[n] @ F[n] @ Gt_fac[n] for n in range(N)]
    return Step(A_new=A_new, dA=dA, g=G, M=M, C=C, Gam=Gam, Gt=Gt_psi, P=P, w=w, f=f, F=F,
                K=K, Psi=Psi, Phi=Phi)


def flat(blocks) -> np.ndarray:
    """Concatenate vec of each block: the parameter vector a (eq. vecV)."""
    return np.concatenate([vec(b) for b in blocks])


def gain_denominator(dA, g, mu: float) -> float:
    """Re(da^H (g + mu da)), the predicted decrease of Section 4.5."""
    da = flat(dA)
    gg = flat(g)
    return float(np.real(np.vdot(da, gg + mu * da)))


# ----------------------------------------------------------------------------
# Normalisation, mu0 and the damping loop (Algorithm 1, Section 4.5)
# ----------------------------------------------------------------------------


def normalize_balanced(A):
    """Spread each component's energy equally over the modes (Algorithm 1,
    normalisation step): lambda_r = prod_n ||a^(n)_r||, a^(n)_r <- a^(n)_r
    lambda_r^(1/N) / ||a^(n)_r||.  Columns with a zero norm are left as they are."""
    N = len(A)
    norms = np.array([np.linalg.norm(a, axis=0) for a in A])   # N x R
    lam = np.prod(norms, axis=0)
    out = []
    for n in range(N):
        s = np.ones_like(lam)
        ok = lam > 0
        s[ok] = lam[ok] ** (1.0 / N) / norms[n, ok]
        out.append(np.asfortranarray(A[n] * s[None, :]))
    return out


def normalize_unit_except_last(A):
    """Unit-norm columns in modes 1..N-1, magnitude carried by mode N (Section 2)."""
    N = len(A)
    out = [a.copy() for a in A]
    for n in range(N - 1):
        nr = np.linalg.norm(out[n], axis=0)
        ok = nr > 0
        out[n][:, ok] /= nr[ok]
        out[N - 1][:, ok] *= nr[ok]
    return [np.asfortranarray(a) for a in out]


def mu0_from_tau(A, tau: float) -> float:
    """mu0 = tau * max diag(H) = tau * max_n max diag Gamma^(n) (eq. mu0)."""
    Gam = gammas(grams(A))
    return float(tau * max(np.max(np.real(np.diag(g))) for g in Gam))


STOP_TOL, STOP_MAX_IT, STOP_MU, STOP_NONFINITE = 0, 1, 2, 3


def fit(Y: np.ndarray, A0, mu0: float, tol: float, max_iters: int, normalize: str = "balanced",
        tau: float = 1e-3, variant: str = "a", trace: bool = False, mu_rule: str = "paper"):
    """Algorithm 1 with the damping of Section 4.5.

    One iteration is one trial step.  A trial is accepted iff the residual
    decreases (equivalently rho > 0, the denominator being positive); then the
    factors are normalised and mu <- mu max(1/3, 1 - (2 rho - 1)^3).  On a
    rejected trial, mu_rule "paper" doubles mu (as Section 4.5 prints it);
    "nielsen" is the rule of the damping paper Section 4.5 cites: mu <- mu nu
    and nu <- 2 nu on a rejection, nu reset to 2 on an acceptance, so that
    consecutive rejections grow mu ever faster.  The fit stops on an accepted
    trial whose relative-error change |eps_prev - eps| is below tol, after
    max_iters trials, or when mu exceeds 1e30.
    """
    if mu_rule not in ("paper", "nielsen"):
        raise ValueError(mu_rule)
    A = [np.array(a, dtype=np.result_type(a, np.float64), order="F") for a in A0]
    normf = {"balanced": normalize_balanced, "unit": normalize_unit_except_last,
             "none": lambda x: x}[normalize]
    if mu0 <= 0:
        mu0 = mu0_from_tau(A, tau)
    mu = mu0
    nu = 2.0
    ynorm = float(np.sqrt(np.sum(np.abs(Y) ** 2)))
    err2 = residual_norm2(Y, A)
    eps = np.sqrt(err2) / ynorm
    hist = []
    reason = STOP_MAX_IT
    it = 0
    accepted = 0
    while it < max_iters:
        st = fast_step(Y, A, mu, variant=variant)
        it += 1
        err2_new = residual_norm2(Y, st.A_new)
        denom = gain_denominator(st.dA, st.g, mu)
        rho = (err2 - err2_new) / denom
        if not np.isfinite(err2_new):
            reason = STOP_NONFINITE
            break
        acc = err2_new < err2
        if trace:
            hist.append(dict(mu=mu, err2=err2, err2_new=err2_new, rho=rho, accepted=acc,
                             dA=st.dA, A=A, gnorm=float(np.linalg.norm(flat(st.g))),
                             Mnorm=float(np.linalg.norm(flat(st.M)))))
        if acc:
            accepted += 1
            A = normf(st.A_new)
            err2 = err2_new
            eps_prev, eps = eps, np.sqrt(err2) / ynorm
            mu = mu * max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
            nu = 2.0
            if abs(eps_prev - eps) < tol:
                reason = STOP_TOL
                break
        elif mu_rule == "paper":
            mu = 2.0 * mu
        else:
            mu = nu * mu
            nu = 2.0 * nu
        if mu > 1e30:
            reason = STOP_MU
            break
    return dict(A=A, iters=it, accepted=accepted, eps=eps, err2=err2, mu=mu, reason=reason,
                hist=hist, mu0=mu0)


# ----------------------------------------------------------------------------
# ALS warm-up (eq. ALS, Section 2; run for a few sweeps after initialisation,
# Section 4.5)
# ----------------------------------------------------------------------------


def als_sweep(Y: np.ndarray, A):
    """One sweep of the ALS rule, modes n = 1..N in turn, each update using the
    factors already updated in this sweep:

        A^(n) <- Y_(n) (Khatri-Rao of A^(k), k != n) (Gamma^(n))^dagger,
        Gamma^(n) = Hadamard_{k != n} A^(k)T A^(k).

    When every factor has full column rank, each Gamma^(n) is positive definite
    (Schur product theorem) and the pseudo-inverse is the inverse; the solve
    goes through a library linear solver on the normal equations.

    Complex tensors (Section 5): the least-squares solution of
    Y_(n) ~ A^(n) KR^T is A^(n) = Y_(n) conj(KR) (KR^T conj(KR))^-1, where
    Y_(n) conj(KR) is the MTTKRP with conjugated factors (Theorem 5.4) and
    KR^T conj(KR) = conj(Gamma^(n)) = Gamma^(n)T with Gamma^(n) the Hadamard
    product of A^(k)H A^(k); for real tensors this is the rule above."""
    cplx = any(np.iscomplexobj(a) for a in A) or np.iscomplexobj(Y)
    dt = np.complex128 if cplx else np.float64
    A = [np.array(a, dtype=dt, copy=True) for a in A]
    for n in range(len(A)):
        M = mttkrp(Y, A, n, conj=cplx)
        G = hadamard_except(grams(A), {n})
        # A^(n) G^T = M  <=>  G A^(n)T = M^T
        A[n] = np.linalg.solve(G, M.T).T
    return A


def als(Y: np.ndarray, A, sweeps: int):
    """`sweeps` ALS sweeps from A; returns the factors and ||Y - Y_hat||^2 after
    each sweep."""
    errs = []
    for _ in range(sweeps):
        A = als_sweep(Y, A)
        errs.append(residual_norm2(Y, A))
    return A, errs


# ----------------------------------------------------------------------------
# SVD initialisation (Section 4.5): the leading R left singular vectors of
# every unfolding
# ----------------------------------------------------------------------------


def canonical_signs(U: np.ndarray) -> np.ndarray:
    """Scale each column by the unit factor that makes its entry of largest
    magnitude (the first one on ties) real and positive: singular vectors are
    defined up to sign (complex: up to a unit complex factor, Section 5)."""
    U = np.array(U, copy=True)
    for r in range(U.shape[1]):
        k = int(np.argmax(np.abs(U[:, r])))
        if np.iscomplexobj(U):
            if U[k, r] != 0:
                U[:, r] = U[:, r] * (np.conj(U[k, r]) / abs(U[k, r]))
        elif U[k, r] < 0:
            U[:, r] = -U[:, r]
    return U


def svd_init(Y: np.ndarray, R: int):
    """A^(n) = the R leading left singular vectors of Y_(n) (columns ordered by
    decreasing singular value, canonical signs), through a library SVD, and the
    singular values."""
    A, S = [], []
    for n in range(Y.ndim):
        U, s, _ = np.linalg.svd(unfold(Y, n), full_matrices=False)
        A.append(canonical_signs(U[:, :R]))
        S.append(s[:R])
    return A, S

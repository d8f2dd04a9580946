"""The plain damped Gauss-Newton step with an explicit Jacobian (Section 3).

a <- a + (J^H J + mu I)^-1 J^H vec(Y - Y_hat), with J the Jacobian of
vec(Y_hat) with respect to a = [vec A^(1); ...; vec A^(N)] (eq. vecV,
Lemma B.1).  Column (n, i, r) of J is vec of the CP term r with factor n
replaced by the unit vector e_i.  This is the definition the fast step must
reproduce; it is only usable on tiny tensors (J has prod(I_n) x R sum(I_n)
entries).  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def jacobian(A) -> np.ndarray:
    N = len(A)
    R = A[0].shape[1]
    dims = [a.shape[0] for a in A]
    dtype = np.result_type(*A)
    cols = []
    for n in range(N):
        for r in range(R):            # vec(A^(n)) is column-major: i fastest, then r
            for i in range(dims[n]):
                t = None
                for k in range(N):
                    if k == n:
                        v = np.zeros(dims[k], dtype=dtype)
                        v[i] = 1.0
                    else:
                        v = A[k][:, r]
                    t = v if t is None else np.multiply.outer(t, v)
                cols.append(t.reshape(-1, order="F"))
    return np.array(cols).T


def model_vec(A) -> np.ndarray:
    dims = [a.shape[0] for a in A]
    R = A[0].shape[1]
    y = np.zeros(dims, dtype=np.result_type(*A))
    for r in range(R):
        t = A[0][:, r]
        for a in A[1:]:
            t = np.multiply.outer(t, a[:, r])
        y = y + t
    return y.reshape(-1, order="F")


def param_vec(A) -> np.ndarray:
    return np.concatenate([a.reshape(-1, order="F") for a in A])


def split_param(x, A):
    out, o = [], 0
    for a in A:
        k = a.size
        out.append(x[o:o + k].reshape(a.shape, order="F"))
        o += k
    return out


def plain_step(y_vec: np.ndarray, A, mu: float):
    """Returns (delta_a blocks, g, H) of the plain damped Gauss-Newton step."""
    J = jacobian(A)
    e = y_vec - model_vec(A)
    H = J.conj().T @ J
    g = J.conj().T @ e
    da = np.linalg.solve(H + mu * np.eye(H.shape[0]), g)
    return split_param(da, A), g, H


def hessian_matvec(A, V):
    """[H v]_n from the block form of Theorem B.2 without forming H:
    real:    V_n Gamma^(n) + sum_{m!=n} A^(n) (Gamma^(n,m) * V_m^T A^(m))
    complex: V_n Gamma^(n)T + sum_{m!=n} A^(n) (Gamma^(n,m)T * V_m^T conj(A^(m)))."""
    N = len(A)
    C = [a.conj().T @ a for a in A]
    R = A[0].shape[1]
    out = []
    for n in range(N):
        Gn = np.ones((R, R), dtype=np.result_type(*C))
        for k in range(N):
            if k != n:
                Gn = Gn * C[k]
        acc = V[n] @ Gn.T
        for m in range(N):
            if m == n:
                continue
            Gnm = np.ones((R, R), dtype=np.result_type(*C))
            for k in range(N):
                if k not in (n, m):
                    Gnm = Gnm * C[k]
            acc = acc + A[n] @ (Gnm.T * (V[m].T @ A[m].conj()))
        out.append(acc)
    return out


def jacobian_matvec(A, V) -> np.ndarray:
    """J v without forming J: sum over n, r of the CP term r with factor n replaced by V_n[:, r]."""
    N = len(A)
    R = A[0].shape[1]
    dims = [a.shape[0] for a in A]
    out = np.zeros(dims, dtype=np.result_type(*A, *V))
    for n in range(N):
        for r in range(R):
            t = None
            for k in range(N):
                v = V[n][:, r] if k == n else A[k][:, r]
                t = v if t is None else np.multiply.outer(t, v)
            out = out + t
    return out.reshape(-1, order="F")

"""Recovery metrics of a CP fit against known factors (host side, NumPy).

Section 6 judges a fit of collinear data by the angle between each original
component a_r^(n) and its estimate after the estimated components have been put
in the original order, and reports MedSAE, 10 log10 of the median over runs of
the squared angle (eq. (equ_MedSAE)).  These functions evaluate results that
the library has already produced; they are not part of the fitting path.

Readings where the paper is silent:
* CP components are determined up to a scale of either sign per mode, so the
  angle is taken between the lines the vectors span: the absolute value of the
  normalised inner product enters the arccos (a^H a_hat for complex factors).
* The order is matched by the assignment that maximises the summed log of the
  per-component congruence prod_n |cos alpha_r^(n)| (Hungarian method).
* The angle is computed as atan2(|a_hat - proj_a(a_hat)| |a|, |a^H a_hat|), the
  same angle as the arccos of the definition, without arccos's loss of
  accuracy for angles near zero.
"""
from __future__ import annotations

import numpy as np

# MedSAE floor: a median squared angle of exactly zero reports this many dB
MEDSAE_FLOOR_DB = -300.0


def _angles(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Angles between the columns of a and b (same shape I x R), in [0, pi/2]."""
    a = np.asarray(a)
    b = np.asarray(b)
    ip = np.sum(np.conj(a) * b, axis=0)
    na2 = np.sum(np.abs(a) ** 2, axis=0)
    perp = b - a * (ip / na2)[None, :]
    s = np.sqrt(np.sum(np.abs(perp) ** 2, axis=0) * na2)
    return np.arctan2(s, np.abs(ip))


def congruence(truth, est) -> np.ndarray:
    """R x R matrix of prod_n |cos| between original component r and estimate q."""
    R = truth[0].shape[1]
    S = np.ones((R, R))
    for a, b in zip(truth, est):
        an = a / np.linalg.norm(a, axis=0)
        bn = b / np.linalg.norm(b, axis=0)
        S *= np.abs(np.conj(an).T @ bn)
    return S


def match_order(truth, est) -> np.ndarray:
    """Permutation p with est[:, p[r]] the estimate of original component r."""
    from scipy.optimize import linear_sum_assignment
    S = congruence(truth, est)
    rows, cols = linear_sum_assignment(-np.log(np.maximum(S, 1e-300)))
    p = np.empty(len(rows), dtype=np.int64)
    p[rows] = cols
    return p


def squared_angular_errors(truth, est) -> np.ndarray:
    """alpha_r^(n)^2 (N x R, radians^2) after matching the component order.

    truth, est: lists of I_n x R factor matrices (the estimate's columns in any
    order, each scaled by any nonzero factor)."""
    p = match_order(truth, est)
    return np.stack([_angles(a, b[:, p]) ** 2 for a, b in zip(truth, est)])


def medsae_db(alpha2_runs) -> np.ndarray:
    """MedSAE in dB per (mode, component) from squared angles of several runs
    (array runs x N x R): 10 log10 of the median over runs."""
    med = np.median(np.asarray(alpha2_runs, dtype=np.float64), axis=0)
    with np.errstate(divide="ignore"):
        db = 10.0 * np.log10(med)
    return np.maximum(db, MEDSAE_FLOOR_DB)


def medsae_summary(alpha2_runs) -> dict:
    """The two averages Section 6 plots: the mean over modes of the first
    component's MedSAE, and the mean over modes and components r >= 2."""
    db = medsae_db(alpha2_runs)
    out = {"medsae_first_db": float(np.mean(db[:, 0]))}
    if db.shape[1] > 1:
        out["medsae_rest_db"] = float(np.mean(db[:, 1:]))
    return out

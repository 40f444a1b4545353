"""Residual certificate for computed eigenpairs of a symmetric operator (the
eigenproblem M Y = Y Omega of Eq. 15, whose lowest roots the Davidson solver
of Sec. III.A, step 4, returns).

TEST INFRASTRUCTURE ONLY: used by the tests to bound how far roots computed
elsewhere (the GPU solver) lie from the exact eigenvalues of the oracle's M,
when M is too large for a dense eigensolver.  It shares no code with the HIP
path.

Given vectors x_1..x_k (any basis of a k-dimensional subspace) and the
oracle's sigma = M x:
  1. Rayleigh-Ritz in their span: Q = orth(X), H = Q^T M Q, H c_j = theta_j c_j,
     u_j = Q c_j, r_j = M u_j - theta_j u_j, e_j = ||r_j||.  By the Cauchy
     interlacing (Poincare) inequality theta_j >= lambda_j, the j-th smallest
     eigenvalue of M: an upper bound that needs no assumption.
  2. Weinstein: M has an eigenvalue in [theta_j - e_j, theta_j + e_j].
  3. Kato-Temple: if the open interval (alpha, beta) around theta_j holds exactly
     one eigenvalue lambda of M, then
        theta_j - e_j^2 / (beta - theta_j) <= lambda <= theta_j + e_j^2 / (theta_j - alpha).
     Here beta = theta_{j+1} - e_{j+1} and alpha = theta_{j-1} + e_{j-1} (the
     neighbours' Weinstein intervals).  Kato-Temple's upper bound theta_j +
     e_j^2 / (theta_j - alpha) is never below theta_j, so step 1's theta_j is
     the upper bound used.  The last vector of the set only
     provides beta for the one before it, so k vectors certify k - 1 roots.

What residuals cannot show: that the solver missed no eigenvalue below or
between the computed ones.  The bound is conditional on that (every lambda_j,
j < k, lies in the j-th Weinstein interval and the intervals are disjoint),
which is checked as far as it can be: disjointness is tested and reported.
"""
from __future__ import annotations

import numpy as np


def rayleigh_ritz(sigma, X):
    """Ritz values, Ritz vectors and residual norms of M in span(X).

    sigma(V[n, dim]) -> M V (rows are vectors); X [k, dim].
    Returns (theta [k] ascending, U [k, dim], res [k])."""
    X = np.asarray(X, dtype=np.float64)
    Qm, _ = np.linalg.qr(X.T)             # dim x k, orthonormal columns
    Q = Qm.T
    S = np.asarray(sigma(Q), dtype=np.float64)
    H = Q @ S.T
    H = 0.5 * (H + H.T)
    theta, C = np.linalg.eigh(H)
    U = C.T @ Q
    R = C.T @ S - theta[:, None] * U
    return theta, U, np.linalg.norm(R, axis=1)


def kato_temple(theta, res):
    """Bounds for the lowest len(theta) - 1 eigenvalues from sorted Ritz values
    and residual norms (steps 2-3 above).

    Returns a dict of arrays over the certified roots: lower, upper (bounds on
    lambda_j), weinstein (e_j), gap (beta_j - theta_j), disjoint (whether the
    Weinstein intervals of roots j and j + 1 are disjoint, which the bound
    requires)."""
    theta = np.asarray(theta, dtype=np.float64)
    res = np.asarray(res, dtype=np.float64)
    k = theta.size
    if k < 2:
        raise ValueError("need at least two Ritz pairs (the last one bounds the gap)")
    if np.any(np.diff(theta) < 0):
        raise ValueError("Ritz values must be sorted ascending")
    n = k - 1
    lower = np.empty(n)
    upper = np.empty(n)
    gap = np.empty(n)
    disjoint = np.empty(n, dtype=bool)
    for j in range(n):
        beta = theta[j + 1] - res[j + 1]
        gap[j] = beta - theta[j]
        disjoint[j] = theta[j] + res[j] < beta
        lower[j] = theta[j] - res[j] ** 2 / gap[j] if gap[j] > 0 else -np.inf
        upper[j] = theta[j]          # Cauchy interlacing (step 1)
        # the Weinstein interval always holds an eigenvalue; never report a
        # lower bound below it
        lower[j] = max(lower[j], theta[j] - res[j])
    return {"lower": lower, "upper": upper, "weinstein": res[:n].copy(), "gap": gap,
            "disjoint": disjoint}


def certify(sigma, X):
    """Rayleigh-Ritz of M on span(X), then Kato-Temple bounds for the lowest
    k - 1 roots.  Returns (theta [k], bounds dict of kato_temple)."""
    theta, _, res = rayleigh_ritz(sigma, X)
    return theta, kato_temple(theta, res)

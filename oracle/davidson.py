"""Textbook block Davidson-Liu eigensolver in FP64 (the oracle's solver).

TEST INFRASTRUCTURE ONLY.

The paper uses a multiroot Davidson solver (Sec. III.A) without giving its
parameters; this module takes the following reading:
  * guesses: unit vectors at the `block` smallest diagonal entries (ties to
    the lower index);
  * each iteration: Rayleigh-Ritz in the current space, residuals
    r_k = W s_k - theta_k V s_k of the lowest `block` Ritz pairs;
  * convergence: every one of the lowest `nroots` roots has
    |theta_k - theta_k(previous)| <= tol_e and ||r_k|| <= tol_r;
  * correction: delta = r / (theta - D) (diagonal preconditioner; entries with
    |theta - D| < 1e-8 use 1e-8 with the same sign), for residuals above tol_r;
  * two Gram-Schmidt passes; a new vector whose norm falls below 1e-10 is
    dropped;
  * restart to the current `block` Ritz vectors when the space would exceed
    max_space (default 8 * block).
"""
from __future__ import annotations

import numpy as np


def davidson(sigma, diag, nroots, block=None, tol_e=1e-8, tol_r=None,
             max_iter=200, max_space=None, precond=None, log=None):
    """Lowest `nroots` eigenpairs of a symmetric operator.

    sigma(X[nvec, dim]) -> [nvec, dim]; diag [dim].  Returns
    (energies [nroots], vectors [nroots, dim], iterations, converged).
    """
    diag = np.asarray(diag, dtype=np.float64)
    dim = diag.size
    block = max(nroots, block or nroots)
    block = min(block, dim)
    if tol_r is None:
        tol_r = np.sqrt(tol_e)
    if max_space is None:
        max_space = 8 * block
    max_space = min(max(max_space, 2 * block), dim)
    order = np.argsort(diag, kind="stable")
    V = np.zeros((block, dim))
    V[np.arange(block), order[:block]] = 1.0
    W = sigma(V)
    theta_old = np.full(block, np.inf)
    it = 0
    converged = False
    while True:
        it += 1
        G = V @ W.T
        G = 0.5 * (G + G.T)
        theta, S = np.linalg.eigh(G)
        nb = min(block, theta.size)
        theta, S = theta[:nb], S[:, :nb]
        X = S.T @ V
        AX = S.T @ W
        R = AX - theta[:, None] * X
        rnorm = np.linalg.norm(R, axis=1)
        de = np.abs(theta[:nroots] - theta_old[:nroots])
        if log is not None:
            log.append({"iter": it, "theta": theta[:nroots].copy(),
                        "rnorm": rnorm[:nroots].copy(), "nvec": V.shape[0]})
        if np.all(de <= tol_e) and np.all(rnorm[:nroots] <= tol_r):
            converged = True
            break
        if it >= max_iter:
            break
        theta_old = np.full(block, np.inf)
        theta_old[:nb] = theta
        sel = [k for k in range(nb) if rnorm[k] > tol_r]
        if not sel:
            sel = list(range(nroots))
        if precond is None:
            den = theta[sel][:, None] - diag[None, :]
            den = np.where(np.abs(den) < 1e-8, np.where(den < 0, -1e-8, 1e-8), den)
            Dx = R[sel] / den
        else:
            Dx = precond(R[sel], theta[sel])
        if V.shape[0] + len(sel) > max_space:
            V, W = X, AX
        new = []
        for d in Dx:
            for _ in range(2):
                d = d - V.T @ (V @ d)
                for q in new:
                    d = d - (q @ d) * q
            nrm = np.linalg.norm(d)
            if nrm > 1e-10:
                new.append(d / nrm)
        if not new:
            # the space is invariant to working precision
            converged = bool(np.all(rnorm[:nroots] <= tol_r))
            break
        Nw = np.array(new)
        V = np.vstack([V, Nw])
        W = np.vstack([W, sigma(Nw)])
    return theta[:nroots], X[:nroots], it, converged

"""Oracle (test infrastructure only): the learned Davidson preconditioner in
plain FP64 NumPy.  Only tests, the smoke check and the benchmark's CPU
baseline import this module; the library never does.

The Davidson correction of Sec. III.A step 4 is, with the diagonal
preconditioner, delta = r / (theta - D) for the residual r = (M - theta) x of
a Ritz pair (theta, x) and the diagonal D of M.  The learned preconditioner
keeps that form and multiplies it, element by element, by (1 + y), where y is
the output of a small multilayer perceptron fed with local information about
the element:

    delta_e = rhat_e * q_e * (1 + y_e),     rhat = r / rms(r),
    q_e     = 1 / (theta - D_e)   with |theta - D_e| floored at 1e-8,
    y_e     = MLP(f_e).

Features f_e (NF = 7), with S = max_p |eps_p| the system's energy scale:
    f0 = (theta - D_e) / S
    f1 = rhat_e
    f2, f3, f4 = eps of the orbitals of the element / S: EA 2p1h element
         (i, a, b): eps_i, eps_a, eps_b; EA 1p element a: 0, eps_a, 0;
         IP 2h1p element (a, i, j): eps_a, eps_i, eps_j; IP 1h element i:
         0, eps_i, 0
    f5 = theta / S
    f6 = 1 for the single-excitation block, 0 for the double block

Network: h1 = tanh(W1 f + b1) (256), h2 = tanh(W2 h1 + b2) (256),
y = w3 . h2 + b3.  Parameters are one flat FP32 vector in the order
W1 [256][7], b1 [256], W2 [256][256], b2 [256], w3 [256], b3 [1].

Training pairs come from the method itself: for a Davidson iterate x_k (unit
norm, sign chosen so that x_k . x* > 0) of a root with converged eigenvector
x*, the ideal correction is the error -(x* - x_k) projected off x_k.  The
target is that direction scaled to the RMS of the diagonal correction:
    t = -e / rms(e) * rms(rhat * q),   e = (x* - x_k) - ((x* - x_k) . x_k) x_k
and the loss is the mean squared difference 0.5 mean_e (delta_e - t_e)^2
over the sampled elements.  Adam (Kingma & Ba) updates the parameters.
"""
from __future__ import annotations

import numpy as np

NF = 7
WIDTH = 256
NPARAM = WIDTH * NF + WIDTH + WIDTH * WIDTH + WIDTH + WIDTH + 1
FLOOR = 1e-8


def unpack(p):
    """Views of the flat parameter vector (see the module docstring)."""
    p = np.asarray(p)
    o = 0
    out = {}
    for name, shape in (("W1", (WIDTH, NF)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)),
                        ("b2", (WIDTH,)), ("w3", (WIDTH,)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def init_params(seed):
    """Scaled Gaussian layers 1-2 (std 1/sqrt(fan_in)); the output layer starts
    at zero, so an untrained network reproduces the diagonal preconditioner."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    v = unpack(p)
    v["W1"][...] = rng.standard_normal((WIDTH, NF)) / np.sqrt(NF)
    v["W2"][...] = rng.standard_normal((WIDTH, WIDTH)) / np.sqrt(WIDTH)
    return p


def forward(p, F):
    """y [n] for features F [n, NF]; returns (y, cache)."""
    v = unpack(p)
    F = np.asarray(F, dtype=np.float64)
    h1 = np.tanh(F @ v["W1"].T + v["b1"])
    h2 = np.tanh(h1 @ v["W2"].T + v["b2"])
    y = h2 @ v["w3"] + v["b3"][0]
    return y, (F, h1, h2)


def backward(p, cache, dy):
    """Gradient of sum_e dy_e * y_e with respect to the flat parameters."""
    v = unpack(p)
    F, h1, h2 = cache
    g = np.zeros(NPARAM)
    gv = unpack(g)
    gv["w3"][...] = h2.T @ dy
    gv["b3"][0] = dy.sum()
    d2 = np.outer(dy, v["w3"]) * (1.0 - h2 ** 2)
    gv["W2"][...] = d2.T @ h1
    gv["b2"][...] = d2.sum(axis=0)
    d1 = (d2 @ v["W2"]) * (1.0 - h1 ** 2)
    gv["W1"][...] = d1.T @ F
    gv["b1"][...] = d1.sum(axis=0)
    return g


def diag_factor(theta, D):
    """q = 1 / (theta - D) with |theta - D| floored at 1e-8 (sign kept)."""
    den = theta - np.asarray(D, dtype=np.float64)
    den = np.where(np.abs(den) < FLOOR, np.where(den < 0, -FLOOR, FLOOR), den)
    return 1.0 / den


def loss_and_grad(p, F, rhat, q, t):
    """0.5 mean (rhat q (1 + y) - t)^2 and its parameter gradient."""
    y, cache = forward(p, F)
    delta = rhat * q * (1.0 + y)
    diff = delta - t
    n = diff.size
    loss = 0.5 * np.dot(diff, diff) / n
    dy = diff * rhat * q / n
    return loss, backward(p, cache, dy)


def adam_step(p, g, m, s, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (p, m, s)."""
    m = beta1 * m + (1.0 - beta1) * g
    s = beta2 * s + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    sh = s / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(sh) + eps), m, s


def element_orbitals(kind, nocc, nvir, eo, ev):
    """(eps_x, eps_p, eps_q, single_flag) for every element of the boundary
    layout: EA [V] ++ [i][a][b]; IP [O] ++ [a][i][j]."""
    eo = np.asarray(eo, dtype=np.float64)
    ev = np.asarray(ev, dtype=np.float64)
    if kind == "ea":
        n1 = nvir
        e1 = (np.zeros(n1), ev.copy(), np.zeros(n1), np.ones(n1))
        ex = np.repeat(eo, nvir * nvir)
        ep = np.tile(np.repeat(ev, nvir), nocc)
        eq = np.tile(ev, nocc * nvir)
    else:
        n1 = nocc
        e1 = (np.zeros(n1), eo.copy(), np.zeros(n1), np.ones(n1))
        ex = np.repeat(ev, nocc * nocc)
        ep = np.tile(np.repeat(eo, nocc), nvir)
        eq = np.tile(eo, nvir * nocc)
    n2 = ex.size
    return (np.concatenate([e1[0], ex]), np.concatenate([e1[1], ep]),
            np.concatenate([e1[2], eq]), np.concatenate([e1[3], np.zeros(n2)]))


def features(kind, nocc, eps, D, theta, r):
    """F [dim, NF] for one residual r of Ritz value theta (module docstring)."""
    eps = np.asarray(eps, dtype=np.float64)
    nvir = eps.size - nocc
    S = np.abs(eps).max()
    ex, ep, eq, single = element_orbitals(kind, nocc, nvir, eps[:nocc], eps[nocc:])
    r = np.asarray(r, dtype=np.float64)
    rhat = r / np.sqrt(np.mean(r * r))
    F = np.empty((r.size, NF))
    F[:, 0] = (theta - np.asarray(D)) / S
    F[:, 1] = rhat
    F[:, 2] = ex / S
    F[:, 3] = ep / S
    F[:, 4] = eq / S
    F[:, 5] = theta / S
    F[:, 6] = single
    return F


def target(x, xstar, rhat, q):
    """Training target for iterate x of the root with eigenvector xstar."""
    x = np.asarray(x, dtype=np.float64)
    xstar = np.asarray(xstar, dtype=np.float64)
    if np.dot(x, xstar) < 0:
        xstar = -xstar
    e = xstar - x
    e = e - np.dot(e, x) * x
    rms_e = np.sqrt(np.mean(e * e))
    return -e / rms_e * np.sqrt(np.mean((rhat * q) ** 2))


def apply(p, kind, nocc, eps, D, theta, r):
    """The learned correction delta for one residual (FP64 reference)."""
    F = features(kind, nocc, eps, D, theta, r)
    y, _ = forward(p, F)
    rhat = F[:, 1]
    return rhat * diag_factor(theta, D) * (1.0 + y)

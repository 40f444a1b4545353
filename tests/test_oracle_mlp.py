"""Pins for the MLP-preconditioner oracle (oracle/mlp.py), CPU only."""
import numpy as np
import pytest

from oracle import mlp


def _small_batch(n=40, seed=0):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((n, mlp.NF))
    rhat = rng.standard_normal(n)
    q = 1.0 / (rng.uniform(0.5, 3.0, n) * rng.choice([-1, 1], n))
    t = rng.standard_normal(n)
    return F, rhat, q, t


def test_gradient_matches_central_differences():
    """Backprop against central finite differences on a sample of parameters
    from every layer (a dropped term or a transposed weight fails here)."""
    p = mlp.init_params(3)
    rng = np.random.default_rng(4)
    v = mlp.unpack(p)
    v["w3"][...] = rng.standard_normal(mlp.WIDTH) * 0.3     # non-zero output layer
    v["b3"][0] = 0.1
    v["b1"][...] = rng.standard_normal(mlp.WIDTH) * 0.1
    F, rhat, q, t = _small_batch()
    loss, g = mlp.loss_and_grad(p, F, rhat, q, t)
    offs = np.cumsum([0, mlp.WIDTH * mlp.NF, mlp.WIDTH, mlp.WIDTH * mlp.WIDTH, mlp.WIDTH,
                      mlp.WIDTH, 1])
    idx = np.concatenate([rng.integers(offs[k], offs[k + 1], 6) for k in range(6)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, F, rhat, q, t)[0] - mlp.loss_and_grad(pm, F, rhat, q, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def test_adam_reaches_quadratic_minimum():
    """Adam on 0.5 |p - c|^2 converges to c (the closed-form minimiser)."""
    c = np.array([1.5, -2.0, 0.25])
    p = np.zeros(3)
    m = np.zeros(3)
    s = np.zeros(3)
    for step in range(1, 3001):
        p, m, s = mlp.adam_step(p, p - c, m, s, step, lr=0.01)
    assert np.abs(p - c).max() < 1e-3


def test_untrained_network_is_the_diagonal_preconditioner():
    """Zero output layer: delta = rhat / (theta - D), the textbook diagonal
    Davidson correction (with the 1e-8 floor)."""
    rng = np.random.default_rng(5)
    O, V = 2, 3
    eps = np.concatenate([np.sort(rng.uniform(-2, -0.3, O)), np.sort(rng.uniform(0.1, 5, V))])
    dim = V + O * V * V
    D = rng.uniform(-1, 8, dim)
    D[4] = 0.7                       # exactly theta: hits the floor
    r = rng.standard_normal(dim)
    p = mlp.init_params(1)
    delta = mlp.apply(p, "ea", O, eps, D, 0.7, r)
    rhat = r / np.sqrt(np.mean(r * r))
    den = 0.7 - D
    den[4] = 1e-8
    assert np.allclose(delta, rhat / den, rtol=1e-14, atol=0)


@pytest.mark.parametrize("kind", ["ea", "ip"])
def test_feature_orbitals_match_explicit_loops(kind):
    O, V = 2, 3
    rng = np.random.default_rng(6)
    eps = np.concatenate([np.sort(rng.uniform(-2, -0.3, O)), np.sort(rng.uniform(0.1, 5, V))])
    eo, ev = eps[:O], eps[O:]
    rows = []
    if kind == "ea":
        rows += [(0.0, ev[a], 0.0, 1.0) for a in range(V)]
        rows += [(eo[i], ev[a], ev[b], 0.0) for i in range(O) for a in range(V) for b in range(V)]
    else:
        rows += [(0.0, eo[i], 0.0, 1.0) for i in range(O)]
        rows += [(ev[a], eo[i], eo[j], 0.0) for a in range(V) for i in range(O) for j in range(O)]
    ref = np.array(rows)
    dim = len(rows)
    D = rng.uniform(0, 5, dim)
    r = rng.standard_normal(dim)
    F = mlp.features(kind, O, eps, D, 0.3, r)
    S = np.abs(eps).max()
    assert np.allclose(F[:, 2:5], ref[:, :3] / S)
    assert np.array_equal(F[:, 6], ref[:, 3])
    assert np.allclose(F[:, 0], (0.3 - D) / S)
    assert np.allclose(F[:, 5], 0.3 / S)
    assert np.isclose(np.mean(F[:, 1] ** 2), 1.0)


def test_target_is_the_projected_error_direction():
    rng = np.random.default_rng(7)
    n = 50
    xstar = rng.standard_normal(n)
    xstar /= np.linalg.norm(xstar)
    x = xstar + 0.1 * rng.standard_normal(n)
    x /= np.linalg.norm(x)
    rhat = rng.standard_normal(n)
    q = rng.uniform(0.2, 1.0, n)
    t = mlp.target(-x, xstar, rhat, q)          # sign of x is irrelevant
    t2 = mlp.target(x, xstar, rhat, q)
    assert abs(np.dot(t2, x)) < 1e-12             # orthogonal to the iterate
    assert np.dot(t2, xstar - x) < 0              # points against the error
    assert np.isclose(np.sqrt(np.mean(t2 ** 2)), np.sqrt(np.mean((rhat * q) ** 2)))
    assert np.allclose(np.abs(np.dot(t, x)), 0, atol=1e-12)

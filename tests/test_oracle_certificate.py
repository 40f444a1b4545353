"""Pins of the residual certificate (oracle/certificate.py) against matrices
whose spectrum is known exactly, and against the dense eigenvalues of the
oracle's explicit ADC matrix (Eq. 15)."""
import numpy as np
import pytest

from oracle.certificate import certify, kato_temple, rayleigh_ritz


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    lam = np.concatenate([[-3.0, -1.0, 0.5, 2.0, 2.7, 4.0], rng.uniform(6.0, 20.0, n - 6)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    M = (Q * lam) @ Q.T
    return 0.5 * (M + M.T), np.sort(lam), Q[:, np.argsort(lam)]


def test_bounds_hold_and_shrink_quadratically():
    M, lam, vec = _matrix(300, 3)
    rng = np.random.default_rng(4)
    k = 6
    noise = rng.standard_normal((k, 300))
    widths, radii = [], []
    for delta in (1e-3, 1e-4):
        X = vec[:, :k].T + delta * noise
        theta, b = certify(lambda V: V @ M, X)
        assert np.all(b["disjoint"])
        for j in range(k - 1):
            assert b["lower"][j] <= lam[j] + 1e-12 and lam[j] <= b["upper"][j] + 1e-12, j
        # Ritz values never lie below the eigenvalues they approximate
        assert np.all(theta[:k] >= lam[:k] - 1e-12)
        widths.append(b["upper"] - b["lower"])
        radii.append(b["weinstein"])
    # ten times smaller errors in the vectors: Weinstein's radius (first order)
    # drops about 10x, the Kato-Temple width (second order) about 100x
    assert np.all(radii[0] / radii[1] > 5) and np.all(radii[0] / radii[1] < 20)
    assert np.all(widths[0] / widths[1] > 50)


def test_exact_vectors_give_tight_bounds():
    M, lam, vec = _matrix(120, 5)
    theta, b = certify(lambda V: V @ M, vec[:, :4].T)
    assert np.max(np.abs(theta - lam[:4])) <= 1e-12
    assert np.max(b["upper"] - b["lower"]) <= 1e-20 + 1e-24


def test_rayleigh_ritz_of_a_rotated_basis():
    """Any basis of the same subspace gives the same Ritz values."""
    M, lam, vec = _matrix(80, 6)
    rng = np.random.default_rng(7)
    X = vec[:, :5].T + 1e-3 * rng.standard_normal((5, 80))
    R = rng.standard_normal((5, 5))
    t1, _, r1 = rayleigh_ritz(lambda V: V @ M, X)
    t2, _, r2 = rayleigh_ritz(lambda V: V @ M, R @ X)
    assert np.allclose(t1, t2, atol=1e-12) and np.allclose(r1, r2, atol=1e-10)


def test_kato_temple_formula_by_hand():
    theta = np.array([1.0, 3.0, 6.0])
    res = np.array([0.1, 0.2, 0.5])
    b = kato_temple(theta, res)
    # root 0: beta = 3 - 0.2 = 2.8, lower = 1 - 0.01 / 1.8; root 1: beta = 5.5
    assert b["lower"][0] == pytest.approx(1.0 - 0.01 / 1.8, rel=1e-15)
    assert b["lower"][1] == pytest.approx(3.0 - 0.04 / 2.5, rel=1e-15)
    assert list(b["upper"]) == [1.0, 3.0]
    # overlapping Weinstein intervals are flagged; the lower bound falls back
    # to Weinstein's
    b = kato_temple(np.array([1.0, 1.05]), np.array([0.1, 0.1]))
    assert not b["disjoint"][0] and b["lower"][0] == pytest.approx(0.9)
    with pytest.raises(ValueError):
        kato_temple(np.array([1.0]), np.array([0.1]))


@pytest.mark.parametrize("kind", ["ea", "ip"])
def test_certificate_on_the_oracle_matrix(kind):
    """Loosely converged vectors of the oracle's own ADC(3) matrix: the
    certified intervals contain the dense eigenvalues of the explicit M."""
    from oracle.radc import RADC
    from synthetic import small_system
    O, V, Q = 3, 7, 20
    eps, B = small_system(O, V, Q, 11)
    ref = RADC(eps, B, O, 3, kind)
    M = ref.explicit()
    lam, vec = np.linalg.eigh(M)
    rng = np.random.default_rng(12)
    X = vec[:, :6].T + 1e-4 * rng.standard_normal((6, M.shape[0]))
    theta, b = certify(ref.sigma, X)
    assert np.all(b["disjoint"])
    scale = max(1.0, float(np.max(np.abs(lam[:6]))))
    for j in range(5):
        assert b["lower"][j] - 1e-12 * scale <= lam[j] <= b["upper"][j] + 1e-12 * scale
    assert np.max(b["upper"] - b["lower"]) < 1e-4 * scale

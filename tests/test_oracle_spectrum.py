"""Pins of the spectral-function oracle (Sec. II propagator and density of
states; Sec. IV photoelectron-spectrum form): its Lorentzian normalisation,
the peak height of an isolated root, the narrow-broadening limit, and the
agreement of the trace of the explicit propagator with the P form when
P = 2 sum_p X_p^2 (both spin components)."""
import numpy as np

from oracle import spectrum


def test_lorentzian_normalisation_and_peak_height():
    e = np.array([-3.0, 1.0, 40.0])
    P = np.array([0.5, 1.5, 2.0])
    eta = 0.05
    w = np.linspace(-2000.0, 2000.0, 4_000_001)
    A = spectrum.spectral_function(w, e, P, eta)
    area = np.trapezoid(A, w)
    # the tails beyond +-2000 carry (eta / pi) (1/(2000 - e)) per root and side
    tail = sum(p * eta / np.pi * (1 / (2000 - x) + 1 / (2000 + x)) for p, x in zip(P, e))
    assert abs(area + tail - P.sum()) < 1e-6
    assert np.all(A > 0)
    # an isolated root: A(w_mu) = P_mu / (pi eta) up to the other roots' tails
    peak = spectrum.spectral_function([40.0], e, P, eta)[0]
    assert abs(peak - 2.0 / (np.pi * eta)) < 1e-4 * peak


def test_narrow_broadening_limit():
    """Integrated against a smooth function, A tends to sum_mu P_mu f(w_mu)."""
    e = np.array([-1.0, 0.3, 2.2])
    P = np.array([1.0, 0.25, 0.75])
    w = np.linspace(-10, 10, 2_000_001)
    f = np.exp(-w ** 2 / 4)
    exact = np.sum(P * np.exp(-e ** 2 / 4))
    errs = []
    for eta in (1e-1, 1e-2, 1e-3):
        A = spectrum.spectral_function(w, e, P, eta)
        errs.append(abs(np.trapezoid(A * f, w) - exact))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 2e-3


def test_trace_of_propagator_equals_P_form():
    rng = np.random.default_rng(4)
    nroots, norb = 5, 7
    X = rng.standard_normal((nroots, norb))
    e = np.sort(rng.uniform(-5, 5, nroots))
    eta = 0.2
    w = np.linspace(-8, 8, 301)
    G = spectrum.propagator(w, e, X, eta)
    # spin orbitals: the two spin components carry the same X, so the trace
    # over spin orbitals doubles the spatial trace; P (both components) = 2 sum X^2
    A_trace = -np.imag(2.0 * np.einsum("kpp->k", G)) / np.pi
    P = 2.0 * np.sum(X ** 2, axis=1)
    assert np.abs(A_trace - spectrum.spectral_function(w, e, P, eta)).max() < 1e-12
    # G is symmetric (real X) and its diagonal matches the explicit matrices
    assert np.abs(G - np.transpose(G, (0, 2, 1))).max() < 1e-14
    d = spectrum.propagator_diagonal(w, e, X, eta)
    brute = np.array([[sum(X[m, p] ** 2 / (wk - e[m] + 1j * eta) for m in range(nroots))
                       for p in range(norb)] for wk in w[:7]])
    assert np.abs(d[:7] - brute).max() < 1e-13

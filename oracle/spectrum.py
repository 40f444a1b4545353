"""Spectral function and propagator from the solver's outputs (the oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.

Definitions (Sec. II, the ADC propagator and density of states, and
Sec. IV, the simulated photoelectron spectrum):
  * G(w) = X (w 1 - Omega)^-1 X^T, evaluated at w + i eta (retarded
    propagator with broadening eta), X[p, mu] the spectroscopic amplitudes,
    Omega the diagonal of transition energies;
  * A(w) = -(1/pi) Im Tr G(w);
  * the photoelectron-spectrum form A(w) = -(1/pi) Im sum_mu P_mu / (w - w_mu + i eta)
    with the spectroscopic factors P_mu.
The library's P (Eq. 50) is the sum over both spin components, P = 2 sum_p X_p^2,
with X one spin component; so the trace over spin orbitals of G built from that
X equals the P form.  Written with numpy complex arithmetic, as the definitions
read.
"""
from __future__ import annotations

import numpy as np


def spectral_function(omega, energies, P, eta):
    """A(w) = -(1/pi) Im sum_mu P_mu / (w - w_mu + i eta) on the grid omega."""
    w = np.asarray(omega, dtype=np.float64)[:, None]
    z = w - np.asarray(energies, dtype=np.float64)[None, :] + 1j * eta
    return -np.imag(np.sum(np.asarray(P, dtype=np.float64)[None, :] / z, axis=1)) / np.pi


def propagator(omega, energies, X, eta):
    """G(w + i eta) = X (w 1 - Omega)^-1 X^T as explicit complex matrices:
    returns [nomega, norb, norb] for X [nroots, norb] (rows: roots)."""
    X = np.asarray(X, dtype=np.float64)
    out = []
    for w in np.asarray(omega, dtype=np.float64):
        D = np.diag(1.0 / (w + 1j * eta - np.asarray(energies, dtype=np.float64)))
        out.append(X.T @ D @ X)
    return np.array(out)


def propagator_diagonal(omega, energies, X, eta):
    """Diagonal G_pp(w + i eta), [nomega, norb] complex."""
    G = propagator(omega, energies, X, eta)
    return np.einsum("kpp->kp", G)

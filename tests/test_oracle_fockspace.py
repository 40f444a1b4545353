"""Pins of the Fock-space ADC construction against quantities the theory fixes.

* Full configuration interaction (exact eigenstates of the same Hamiltonian):
  ADC(n) attachment/ionisation energies and spectroscopic factors of the main
  state, and the ground-state energy through order n, differ from the exact
  ones by O(lam^(n+1)) when the perturbation is scaled by lam (Eq. 4: the
  approximation is exact through order n).  Scaling B by sqrt(lam) scales V by
  lam with the Fock matrix fixed, so halving lam must divide the error by
  2^(n+1).  A dropped or mis-signed term at any order <= n breaks this.
* Koopmans limit (B = 0): M is diagonal with eps_a / -eps_i (1p/1h) and the
  zeroth-order 2p1h/2h1p energies; each main state has unit spin-orbital
  strength.
* Hermiticity of M; irrelevance of triples for n <= 3 (the statement after
  Eq. 12 that only singles through n and doubles through n-1 are needed).
"""
import numpy as np
import pytest

from oracle.fockspace import FockSpaceADC, op_matrix
from synthetic import small_system


def _exact(fs, kind, nstate=2):
    eN, vN = np.linalg.eigh(fs.HN)
    eX, vX = np.linalg.eigh(fs.HX)
    g = vN[:, 0]
    P = 0.0
    for p in range(fs.m):
        ap = op_matrix([(p, 1 if kind == "ea" else 0)], fs.secN, fs.secX)
        P += np.sum((vX[:, :nstate].T @ (ap @ g)) ** 2)
    return eX[0] - eN[0], eN[0], P


@pytest.mark.parametrize("kind", ["ea", "ip"])
@pytest.mark.parametrize("order", [2, 3])
def test_error_order_against_full_ci(kind, order):
    eps, B = small_system(2, 3, 8, seed=1)
    errs = []
    for lam in (0.02, 0.01):
        fs = FockSpaceADC(eps, B, 2, order, kind, lam=lam)
        w, v = np.linalg.eigh(fs.M)
        P_adc = np.sum((fs.T @ v[:, :2]) ** 2)       # degenerate Ms = +-1/2 pair
        om, e0, P = _exact(fs, kind)
        errs.append((w[0] - om, sum(fs.E0) - e0, P_adc - P))
    expect = 2.0 ** (order + 1)
    for q in range(3):
        ratio = errs[0][q] / errs[1][q]
        assert abs(ratio - expect) < 0.15 * expect, (q, ratio, errs)
    # and the error is genuinely small at lam = 0.01
    assert abs(errs[1][0]) < 1e-6


@pytest.mark.parametrize("kind", ["ea", "ip"])
def test_koopmans_limit(kind):
    eps, B = small_system(2, 3, 6, seed=2)
    fs = FockSpaceADC(eps, B * 0.0, 2, 3, kind)
    M = fs.M
    assert np.abs(M - np.diag(np.diag(M))).max() < 1e-14
    eso = np.repeat(eps, 2)
    for c, (cl, lab) in enumerate(fs.labels):
        if cl == "1":
            ref = eso[lab] if kind == "ea" else -eso[lab]
        elif kind == "ea":
            A, Bq, I = lab
            ref = eso[A] + eso[Bq] - eso[I]
        else:
            I, J, A = lab
            ref = eso[A] - eso[I] - eso[J]
        assert abs(M[c, c] - ref) < 1e-13
    # one unit of strength per 1p/1h spin orbital, none in 2p1h/2h1p
    assert np.allclose(np.sum(fs.T ** 2, axis=0), (fs.cls == 0).astype(float))


@pytest.mark.parametrize("kind", ["ea", "ip"])
def test_symmetric_and_triples_irrelevant(kind):
    eps, B = small_system(2, 3, 8, seed=3)
    a = FockSpaceADC(eps, B, 2, 3, kind)
    b = FockSpaceADC(eps, B, 2, 3, kind, ranks=(1, 2, 3))
    assert np.abs(a.M - a.M.T).max() < 1e-13
    assert np.abs(a.M - b.M).max() < 1e-12
    assert np.abs(a.T - b.T).max() < 1e-12


def test_mp2_energy_closed_form():
    """Second-order energy equals the closed-shell MP2 formula."""
    eps, B = small_system(2, 3, 8, seed=4)
    fs = FockSpaceADC(eps, B, 2, 2, "ea")
    O = 2
    eri = np.einsum("Qpq,Qrs->pqrs", B, B)
    e2 = 0.0
    n = eps.size
    for i in range(O):
        for j in range(O):
            for a in range(O, n):
                for b in range(O, n):
                    iajb, ibja = eri[i, a, j, b], eri[i, b, j, a]
                    e2 += iajb * (2 * iajb - ibja) / (eps[i] + eps[j] - eps[a] - eps[b])
    assert abs(fs.E0[2] - e2) < 1e-13


def test_unrestricted_closed_shell_limit():
    """Beta set equal to the alpha set: the unrestricted construction gives the
    closed-shell matrices exactly."""
    eps, B = small_system(2, 3, 8, seed=5)
    for kind in ("ea", "ip"):
        a = FockSpaceADC(eps, B, 2, 3, kind)
        b = FockSpaceADC(eps, B, 2, 3, kind, eps_b=eps, B_b=B, nocc_b=2)
        assert a.labels == b.labels
        assert np.abs(a.M - b.M).max() < 1e-12
        assert np.abs(a.T - b.T).max() < 1e-12


@pytest.mark.parametrize("kind", ["ea", "ip"])
@pytest.mark.parametrize("order", [2, 3])
def test_unrestricted_error_order_against_full_ci(kind, order):
    """Open-shell doublet (2 alpha, 1 beta electrons in 4 orbitals): ADC(n)
    energies and the main state's strength differ from full CI by
    O(lam^(n+1)), as for the closed shell."""
    from synthetic import draw_system_u
    ea, eb, Ba, Bb = draw_system_u(2, 1, 4, 8, seed=6)
    errs = []
    for lam in (0.02, 0.01):
        fs = FockSpaceADC(ea, Ba, 2, order, kind, lam=lam, eps_b=eb, B_b=Bb, nocc_b=1)
        assert np.abs(fs.M - fs.M.T).max() < 1e-13
        w, v = np.linalg.eigh(fs.M)
        P_adc = np.sum((fs.T @ v[:, :1]) ** 2)
        om, e0, P = _exact(fs, kind, nstate=1)
        errs.append((w[0] - om, sum(fs.E0) - e0, P_adc - P))
    expect = 2.0 ** (order + 1)
    for q in range(3):
        ratio = errs[0][q] / errs[1][q]
        assert abs(ratio - expect) < 0.15 * expect, (q, ratio, errs)
    assert abs(errs[1][0]) < 1e-6

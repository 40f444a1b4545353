"""Pins of the unrestricted EA/IP-ADC(2) oracle (oracle/uadc.py).

* Against the Fock-space construction with an unrestricted reference (Eqs.
  7-10 evaluated literally, itself pinned against full CI): the whole matrix
  element by element after the map between the two bases (a permutation and
  signs from the order of the two like indices), the transition moments
  (Eqs. 8/10) row by row, for open-shell doublets and a triplet.
* Closed-shell limit (beta set = alpha set): every eigenvalue of the
  spin-adapted restricted oracle (oracle/radc.py) is an eigenvalue here, and
  its Eq. 50 factor is the sum over the Ms = +-1/2 pair.
* sigma = M Y and the diagonal against the explicit matrix; the layout's
  dimension formula.
"""
import numpy as np
import pytest

from oracle.fockspace import FockSpaceADC
from oracle.uadc import UADC2
from synthetic import draw_system_u, small_system


def _alpha_first(fs, u):
    """Map an interleaved spin orbital P = 2p + s to (space, alpha-first index)."""
    def m(P):
        p, s = divmod(P, 2)
        if P in fs.occ:
            return "o", (p if s == 0 else u.Oa + p)
        return "v", (p - u.Oa if s == 0 else u.Va + (p - u.Ob))
    return m


def _basis_map(fs, u):
    """For each Fock-space basis label: (index in the oracle's vector, sign), or
    None for spin combinations outside both sectors."""
    m = _alpha_first(fs, u)
    pos = {tuple(r): k for k, r in enumerate(u.idx2.tolist())}
    out = []
    for cl, lab in fs.labels:
        if cl == "1":
            out.append((m(lab)[1], 1.0))
            continue
        if u.kind == "ea":
            a, b, i = lab
            x, p, q = m(i)[1], m(a)[1], m(b)[1]
        else:
            i, j, a = lab
            x, p, q = m(a)[1], m(i)[1], m(j)[1]
        sgn = 1.0
        if p > q:
            p, q, sgn = q, p, -1.0
        k = pos.get((x, p, q))
        out.append(None if k is None else (u.n1 + k, sgn))
    return out


def _compare(fs, u):
    bm = _basis_map(fs, u)
    keep = [c for c, r in enumerate(bm) if r is not None]
    drop = [c for c, r in enumerate(bm) if r is None]
    # the dropped (|dMs| = 3/2) states do not couple to the kept ones
    if drop:
        assert np.abs(fs.M[np.ix_(keep, drop)]).max() < 1e-13
    idx = np.array([bm[c][0] for c in keep])
    sgn = np.array([bm[c][1] for c in keep])
    assert sorted(idx.tolist()) == list(range(u.dim))
    Mf = fs.M[np.ix_(keep, keep)] * sgn[:, None] * sgn[None, :]
    Mu = u.explicit()[np.ix_(idx, idx)]
    scale = np.abs(Mf).max()
    assert np.abs(Mf - Mu).max() <= 1e-12 * scale
    # transition moments: rows are spin orbitals, alpha-first (alpha orbitals
    # 0..N-1, then beta) in the oracle
    E = np.zeros((u.dim, u.dim))
    E[idx, np.arange(len(idx))] = sgn
    Tu = u.spec_amplitudes(E.T).T                  # [2N][kept Fock columns]
    Tf = fs.T[:, keep]
    rows = [(P % 2) * u.N + P // 2 for P in range(2 * u.N)]
    assert np.abs(Tf - Tu[rows]).max() <= 1e-12 * max(1.0, np.abs(Tf).max())


@pytest.mark.parametrize("kind", ["ea", "ip"])
@pytest.mark.parametrize("occ", [(2, 1), (3, 2), (3, 1)])
def test_matches_fock_space_unrestricted(kind, occ):
    Oa, Ob = occ
    N = 5
    ea, eb, Ba, Bb = draw_system_u(Oa, Ob, N, 9, seed=20 + Oa + 3 * Ob)
    fs = FockSpaceADC(ea, Ba, Oa, 2, kind, eps_b=eb, B_b=Bb, nocc_b=Ob)
    u = UADC2(ea, eb, Ba, Bb, Oa, Ob, kind)
    _compare(fs, u)


@pytest.mark.parametrize("kind", ["ea", "ip"])
def test_closed_shell_limit_contains_restricted_roots(kind):
    from oracle.radc import RADC
    O, V, Q = 3, 6, 15
    eps, B = small_system(O, V, Q, 31)
    u = UADC2(eps, eps, B, B, O, O, kind)
    r = RADC(eps, B, O, 2, kind)
    wu, vu = np.linalg.eigh(u.explicit())
    wr, vr = np.linalg.eigh(r.explicit())
    Pu = u.spec_factors(vu.T)
    Pr = r.spec_factors(vr.T)
    for w, P in zip(wr, Pr):
        hit = np.abs(wu - w) < 1e-9 * max(1.0, abs(w))
        assert hit.sum() >= 2, w          # the Ms = +-1/2 pair (quartets may add more)
        # the doublet pair carries the restricted factor (factor 2 of Eq. 50)
        if hit.sum() == 2:
            assert abs(Pu[hit].sum() - P) <= 1e-9 * max(1.0, abs(P))


@pytest.mark.parametrize("kind", ["ea", "ip"])
def test_sigma_diag_and_dimension(kind):
    Oa, Ob, N = 4, 2, 9
    ea, eb, Ba, Bb = draw_system_u(Oa, Ob, N, 20, seed=41)
    u = UADC2(ea, eb, Ba, Bb, Oa, Ob, kind)
    Va, Vb = N - Oa, N - Ob
    if kind == "ea":
        dim = Va + Vb + Oa * Va * (Va - 1) // 2 + Ob * Va * Vb + Oa * Va * Vb + Ob * Vb * (Vb - 1) // 2
    else:
        dim = Oa + Ob + Va * Oa * (Oa - 1) // 2 + Vb * Oa * Ob + Va * Oa * Ob + Vb * Ob * (Ob - 1) // 2
    assert u.dim == dim
    M = u.explicit()
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    assert np.abs(np.diag(M) - u.diag()).max() <= 1e-13 * np.abs(M).max()
    X = np.random.default_rng(42).standard_normal((3, u.dim))
    assert np.abs(u.sigma(X) - X @ M.T).max() <= 1e-12 * np.abs(M).max()
    # the two spin sectors do not couple
    n1a = Va if kind == "ea" else Oa
    sec = np.zeros(u.dim, dtype=bool)
    sec[:n1a] = True
    if kind == "ea":
        n_aaa, n_bab = Oa * Va * (Va - 1) // 2, Ob * Va * Vb
        off = Va + Vb
    else:
        n_aaa, n_bab = Va * Oa * (Oa - 1) // 2, Vb * Oa * Ob
        off = Oa + Ob
    sec[off:off + n_aaa + n_bab] = True
    assert np.abs(M[np.ix_(sec, ~sec)]).max() == 0.0

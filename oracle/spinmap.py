"""Map between the spin-adapted Z basis and spin-orbital ADC vectors.

TEST INFRASTRUCTURE ONLY.  Used to pin the spin-adapted oracle against the
Fock-space construction: M_Z must equal U^T M_so U, where U sends a Z-basis
vector to the spin-orbital ADC basis of ``fockspace.FockSpaceADC``.

Spin adaptation (Sec. III.B): an EA state with an alpha electron attached has
spin-orbital amplitudes
  Y(A)     = d(sA, alpha) Y1_a
  Y(A,B,I) = d(sA, alpha) d(sB, sI) Y2_abi - d(sB, alpha) d(sA, sI) Y2_bai,
the IP analogue (alpha electron removed) being
  Y(I)     = d(sI, alpha) Y1_i
  Y(I,J,A) = d(sI, alpha) d(sJ, sA) Y2_ija - d(sJ, alpha) d(sI, sA) Y2_jia,
which reproduces the element map of Eqs. 20-27 (mixed-spin blocks carry the
spatial amplitude, the same-spin block its antisymmetrised combination).
Y = S^{-1/2} Z with the pair metric of Eq. 48.
"""
from __future__ import annotations

import numpy as np

from .fockspace import op_matrix
from .radc import ALI, BEI


def z_to_spin_orbital(fs, kind, O, V):
    """Matrix U [dim_so, dim_Z] for a FockSpaceADC object."""
    labels = fs.labels
    col = {lab: c for c, lab in enumerate(labels)}
    n1 = V if kind == "ea" else O
    dimz = (V + O * V * V) if kind == "ea" else (O + O * O * V)
    U = np.zeros((len(labels), dimz))
    # 1p / 1h
    for x in range(n1):
        P = 2 * (x + (O if kind == "ea" else 0))      # alpha spin orbital
        U[col[("1", P)], x] = 1.0

    def put(lab_fn, x, y, z, coef, zcol):
        # spin-orbital amplitude of (x,y,z) labelled state, antisymmetric in x,y
        A, Bq, C = lab_fn(x, y, z)
        if A == Bq:
            return
        if A < Bq:
            U[col[("2", (A, Bq, C))], zcol] += coef
        else:
            U[col[("2", (Bq, A, C))], zcol] -= coef

    if kind == "ea":
        def zidx(i, a, b):
            return V + (i * V + a) * V + b
        for i in range(O):
            for a in range(V):
                for b in range(V):
                    # Y2_abi in terms of Z: ALI Z_abi + BEI Z_bai
                    for (zc, w) in ((zidx(i, a, b), ALI), (zidx(i, b, a), BEI)):
                        aa, bb, ii = O + a, O + b, i
                        # + d(sA,alpha) d(sB,sI) Y2_abi
                        for s in (0, 1):
                            put(lambda x, y, z: (x, y, z), 2 * aa, 2 * bb + s, 2 * ii + s, w, zc)
                        # - d(sB,alpha) d(sA,sI) Y2_bai contributes to Y(A,B,I)
                        # with A=(b, s), B=(a, alpha): that is the same state set
    else:
        def zidx(a, i, j):
            return O + (a * O + i) * O + j
        for a in range(V):
            for i in range(O):
                for j in range(O):
                    for (zc, w) in ((zidx(a, i, j), ALI), (zidx(a, j, i), BEI)):
                        for s in (0, 1):
                            put(lambda x, y, z: (x, y, z), 2 * i, 2 * j + s, 2 * (O + a) + s, w, zc)
    return U


def s2_operator(sec):
    """Total spin S^2 on a determinant sector (spin orbital P = 2p + s)."""
    m = sec.m
    n = m // 2
    Sp = np.zeros((sec.dim, sec.dim))
    Sz = np.zeros(sec.dim)
    for p in range(n):
        Sp += op_matrix([(2 * p, 1), (2 * p + 1, 0)], sec, sec)
    for k, d in enumerate(sec.dets):
        na = sum((d >> (2 * p)) & 1 for p in range(n))
        nb = sum((d >> (2 * p + 1)) & 1 for p in range(n))
        Sz[k] = 0.5 * (na - nb)
    Sm = Sp.T
    return Sm @ Sp + np.diag(Sz * (Sz + 1.0))

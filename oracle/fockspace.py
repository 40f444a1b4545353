"""Fock-space construction of the EA/IP-ADC(n) matrices from their definitions.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module.

This is the plainest possible reading of the effective-Liouvillean ADC
equations (Sec. II, Eqs. 5-14): every operator is a dense matrix on the
determinant space of a fixed particle number, every perturbation order is a
separate matrix, and the matrix elements of M and T are read off directly.
No hand-derived ADC working equation is used anywhere in this file.

Spin orbitals: spatial orbital p with spin s (0 = alpha, 1 = beta) is spin
orbital P = 2p + s.  Occupied spatial orbitals come first.  Determinants are
bit masks; a_P carries the Jordan-Wigner sign (-1)^(number of occupied spin
orbitals below P).

Hamiltonian (canonical-HF reading of a synthetic system): the Fock matrix is
diag(eps) by construction, so the core Hamiltonian is
h_pq = eps_p delta_pq - sum_k [2 (pq|kk) - (pk|kq)], and the two-electron
integrals are (pq|rs) = sum_Q B^Q_pq B^Q_rs (Eq. 38).  Moller-Plesset
partitioning (Sec. II, Eq. 14 and the text after it): H0 = sum_P eps_P a_P^+ a_P
and V = H - H0; the perturbation parameter lam multiplies V.

Effective Hamiltonian (Eq. 11): Ht = exp(-A) H exp(A) with A = sum_k lam^k A_k,
A_k = T^(k) - T^(k)+.  Amplitudes (Eqs. 13-14): at order k, the singles and
doubles projections of Ht^(k) vanish, which gives
t_mu^(k) = -<Phi_mu| Ht^(k)[A_k = 0] |Phi> / D_mu.  Following the statement
after Eq. 12, singles are solved through order n and doubles through order
n-1 (`ranks` may add higher ranks; they do not change M or T for n <= 3).

EA matrix (Eq. 7) with h^(0)+ = a_a^+ and h^(1)+ = a_b^+ a_a^+ a_i: because
h_mu|Phi> = 0, the anticommutator expectation value reduces to
M_mu,nu = <Psi_mu|Ht|Psi_nu> - delta_mu,nu <Phi|Ht|Phi>, Psi_nu = h_nu^+ |Phi>.
The order of a contribution is k + l + m where k, m are the operator classes,
so the (11, 12, 22) blocks take Ht through orders (n, n-1, n-2).
EA transition moments (Eq. 8): T_p,nu = <Phi| at_p |Psi_nu> with the class of
nu added to the order of at_p (Eq. 12).

IP matrix (Eq. 9) with h^(0)+ = a_i and h^(1)+ = a_a^+ a_j a_i: the
expectation value gives M_- = E0 delta - <Psi|Ht|Psi>, whose eigenvalues are
E^N - E^(N-1).  This module returns K = -M_-, whose eigenvalues are the
ionisation energies (positive), as the library does.  IP transition moments
(Eq. 10): T_p,nu = <Psi_nu| at_p |Phi>.
"""
from __future__ import annotations

from itertools import combinations
from math import factorial

import numpy as np


# ---------------------------------------------------------------------------
# integrals in the spin-orbital basis
# ---------------------------------------------------------------------------

def spatial_integrals(eps, B):
    """(pq|rs) from the DF factors (Eq. 38) and the core Hamiltonian h_pq."""
    eri = np.einsum("Qpq,Qrs->pqrs", B, B)
    return eri


def core_hamiltonian(eps, eri, nocc):
    """h with Fock matrix f = h + sum_k [2(pq|kk) - (pk|kq)] equal to diag(eps)."""
    o = slice(0, nocc)
    J = np.einsum("pqkk->pq", eri[:, :, o, o])
    K = np.einsum("pkkq->pq", eri[:, o, o, :])
    return np.diag(eps) - (2.0 * J - K)


def spin_orbital_tensors(eps, B, nocc, eri=None):
    """Spin-orbital eps_P, h_PQ and <PQ|RS> = (pr|qs) delta(sP,sR) delta(sQ,sS).

    `eri` (chemists' (pq|rs)) replaces the DF product when given.
    """
    n = eps.size
    if eri is None:
        eri = spatial_integrals(eps, B)
    h = core_hamiltonian(eps, eri, nocc)
    m = 2 * n
    eps_so = np.repeat(eps, 2)
    h_so = np.zeros((m, m))
    g_so = np.zeros((m, m, m, m))
    for s in range(2):
        h_so[s::2, s::2] = h
    for s1 in range(2):
        for s2 in range(2):
            # <P Q | R S> with P=(p,s1), Q=(q,s2), R=(r,s1), S=(s,s2)  -> (pr|qs)
            g_so[s1::2, s2::2, s1::2, s2::2] = eri.transpose(0, 2, 1, 3)
    return eps_so, h_so, g_so


def spin_orbital_tensors_u(eps_a, eps_b, B_a, B_b, nocc_a, nocc_b):
    """Unrestricted (open-shell) reference: spin-orbital eps_P, h_PQ and
    <PQ|RS> = (pr|qs)_{sP sQ} delta(sP,sR) delta(sQ,sS), where
    (pq|rs)_{st} = sum_Q B_s^Q_pq B_t^Q_rs (Eq. 38 for each pair of spins).

    Canonical-UHF reading of a synthetic system: each spin's Fock matrix
    f^s_pq = h^s_pq + sum_t sum_{k occ in t} (pq|kk)_{st} - sum_{k occ in s} (pk|kq)_{ss}
    is diag(eps_s) by construction, which fixes h^s (the one-electron operator
    then depends on the spin, as a UHF Fock operator does)."""
    eps = (np.asarray(eps_a, dtype=np.float64), np.asarray(eps_b, dtype=np.float64))
    B = (np.asarray(B_a, dtype=np.float64), np.asarray(B_b, dtype=np.float64))
    nocc = (nocc_a, nocc_b)
    n = eps[0].size
    eri = {(s, t): np.einsum("Qpq,Qrs->pqrs", B[s], B[t]) for s in range(2) for t in range(2)}
    m = 2 * n
    eps_so = np.zeros(m)
    h_so = np.zeros((m, m))
    g_so = np.zeros((m, m, m, m))
    for s in range(2):
        eps_so[s::2] = eps[s]
        J = sum(np.einsum("pqkk->pq", eri[s, t][:, :, :nocc[t], :nocc[t]]) for t in range(2))
        K = np.einsum("pkkq->pq", eri[s, s][:, :nocc[s], :nocc[s], :])
        h_so[s::2, s::2] = np.diag(eps[s]) - J + K
    for s1 in range(2):
        for s2 in range(2):
            g_so[s1::2, s2::2, s1::2, s2::2] = eri[s1, s2].transpose(0, 2, 1, 3)
    return eps_so, h_so, g_so


# ---------------------------------------------------------------------------
# determinant spaces and second-quantised operators
# ---------------------------------------------------------------------------

class Sector:
    """All determinants with `nel` electrons in `m` spin orbitals."""

    def __init__(self, m: int, nel: int):
        self.m, self.nel = m, nel
        self.dets = [sum(1 << p for p in c) for c in combinations(range(m), nel)]
        self.index = {d: i for i, d in enumerate(self.dets)}
        self.dim = len(self.dets)


def _apply(ops, det):
    """Apply a product of operators (rightmost first) to a determinant.

    ops is a list of (P, dagger).  Returns (sign, det) or None.
    """
    sign = 1
    for p, dag in reversed(ops):
        occ = (det >> p) & 1
        if dag == occ:  # create on occupied or annihilate empty
            return None
        if bin(det & ((1 << p) - 1)).count("1") & 1:
            sign = -sign
        det ^= 1 << p
    return sign, det


def op_matrix(ops, src: Sector, dst: Sector):
    """Dense matrix of an operator string from sector src to sector dst."""
    M = np.zeros((dst.dim, src.dim))
    for j, d in enumerate(src.dets):
        r = _apply(ops, d)
        if r is not None:
            M[dst.index[r[1]], j] += r[0]
    return M


def hamiltonian(h_so, g_so, sec: Sector):
    """H = sum h_PQ a+_P a_Q + 1/2 sum <PQ|RS> a+_P a+_Q a_S a_R on a sector.

    Uses a+_P a+_Q a_S a_R = E_PR E_QS - delta_QR E_PS with E_PQ = a+_P a_Q.
    """
    from scipy import sparse
    m = h_so.shape[0]
    E = {}
    for P in range(m):
        for Q in range(m):
            E[P, Q] = sparse.csr_matrix(op_matrix([(P, 1), (Q, 0)], sec, sec))
    H = sparse.csr_matrix((sec.dim, sec.dim))
    for P in range(m):
        for S in range(m):
            c = h_so[P, S] - 0.5 * np.einsum("qq->", g_so[P, :, :, S])
            if c != 0.0:
                H = H + c * E[P, S]
    for P in range(m):
        for R in range(m):
            F = sparse.csr_matrix((sec.dim, sec.dim))
            for Q in range(m):
                for S in range(m):
                    c = g_so[P, Q, R, S]
                    if c != 0.0:
                        F = F + c * E[Q, S]
            if F.nnz:
                H = H + 0.5 * (E[P, R] @ F)
    return H.toarray()


# ---------------------------------------------------------------------------
# truncated power series in the perturbation parameter
# ---------------------------------------------------------------------------

def s_mul(X, Y, n):
    """Product of two series [X0, X1, ...] truncated after order n."""
    out = []
    for k in range(n + 1):
        acc = None
        for i in range(k + 1):
            if i < len(X) and k - i < len(Y) and X[i] is not None and Y[k - i] is not None:
                t = X[i] @ Y[k - i]
                acc = t if acc is None else acc + t
        out.append(acc)
    return out


def s_exp(A, n, dim):
    """exp(A) for a series A with A[0] = 0, truncated after order n."""
    out = [np.eye(dim)] + [None] * n
    term = [np.eye(dim)] + [None] * n
    for j in range(1, n + 1):
        term = s_mul(term, A, n)
        for k in range(n + 1):
            if term[k] is not None:
                add = term[k] / factorial(j)
                out[k] = add if out[k] is None else out[k] + add
    return out


def _coef(S, k, dim):
    return S[k] if (k < len(S) and S[k] is not None) else np.zeros((dim, dim))


# ---------------------------------------------------------------------------
# the ADC construction
# ---------------------------------------------------------------------------

class FockSpaceADC:
    """EA/IP-ADC(n) matrices of a closed-shell or (with eps_b, B_b, nocc_b) an
    open-shell unrestricted reference, built in Fock space.

    Parameters: eps [N], B [Naux, N, N], nocc, order n (2 or 3), kind "ea"/"ip";
    for an unrestricted reference eps, B, nocc are the alpha ones and eps_b,
    B_b, nocc_b the beta ones.
    Attributes after construction:
      M       spin-orbital ADC matrix (EA: M_+, IP: K = -M_-), symmetric
      T       transition moments [2N, dim]
      labels  basis labels: ("1", P) or ("2", (A, B, I)) for EA (a<b virtual),
              ("1", I) or ("2", (I, J, A)) for IP (I<J occupied)
      E0      [E^(0), E^(1), ..., E^(n)] ground-state energy by order
      amps    {k: {"t1": [2N,2N] array, "t2": {(I,J,A,B): t}}}
    """

    def __init__(self, eps, B, nocc, order, kind, ranks=(1, 2), lam=1.0, eri=None,
                 eps_b=None, B_b=None, nocc_b=None):
        self.eps = np.asarray(eps, dtype=np.float64)
        self.B = None if B is None else np.asarray(B, dtype=np.float64) * np.sqrt(lam)
        eri = None if eri is None else np.asarray(eri, dtype=np.float64) * lam
        self.nocc, self.order, self.kind = nocc, order, kind
        n = self.eps.size
        self.nmo = n
        self.m = m = 2 * n
        if eps_b is None:
            # closed shell: spin orbitals 0 .. 2 nocc - 1 occupied
            self.occ = list(range(2 * nocc))
            self.vir = list(range(2 * nocc, m))
            self.eps_so, h_so, g_so = spin_orbital_tensors(self.eps, self.B, nocc, eri)
        else:
            # unrestricted reference: nocc alpha (P = 2p, p < nocc) and nocc_b
            # beta (P = 2p + 1, p < nocc_b) spin orbitals occupied
            Bb = np.asarray(B_b, dtype=np.float64) * np.sqrt(lam)
            self.occ = sorted([2 * p for p in range(nocc)] + [2 * p + 1 for p in range(nocc_b)])
            self.vir = [P for P in range(m) if P not in self.occ]
            self.eps_so, h_so, g_so = spin_orbital_tensors_u(self.eps, eps_b, self.B, Bb,
                                                             nocc, nocc_b)
        nel = len(self.occ)
        self.secN = Sector(m, nel)
        self.secX = Sector(m, nel + 1 if kind == "ea" else nel - 1)
        self.HN = hamiltonian(h_so, g_so, self.secN)
        self.HX = hamiltonian(h_so, g_so, self.secX)
        self.H0N = np.diag([self._h0(d) for d in self.secN.dets])
        self.H0X = np.diag([self._h0(d) for d in self.secX.dets])
        self.phi = np.zeros(self.secN.dim)
        self.ref = sum(1 << p for p in self.occ)
        self.phi[self.secN.index[self.ref]] = 1.0
        self._solve_amplitudes(ranks)
        self._build_matrices()

    # zeroth-order energy of a determinant
    def _h0(self, det):
        return sum(self.eps_so[p] for p in range(self.m) if (det >> p) & 1)

    def _excitations(self, rank):
        """Excitation strings a+_A1 ... a+_Ar a_Ir ... a_I1 with A1<..<Ar, I1<..<Ir."""
        out = []
        for I in combinations(self.occ, rank):
            for A in combinations(self.vir, rank):
                ops = [(a, 1) for a in A] + [(i, 0) for i in reversed(I)]
                D = sum(self.eps_so[a] for a in A) - sum(self.eps_so[i] for i in I)
                out.append((I, A, ops, D))
        return out

    def _A_matrix(self, amps_k, sec):
        """A_k = T^(k) - T^(k)+ on a sector."""
        A = np.zeros((sec.dim, sec.dim))
        for (ops, t) in amps_k:
            if t != 0.0:
                X = op_matrix(ops, sec, sec)
                A += t * (X - X.T)
        return A

    def _Ht(self, Aser, H0, H, n):
        """Effective Hamiltonian series exp(-A) (H0 + lam V) exp(A) through order n."""
        dim = H0.shape[0]
        Hs = [H0, H - H0]
        Ep = s_exp(Aser, n, dim)
        Em = s_exp([None if a is None else -a for a in Aser], n, dim)
        return s_mul(s_mul(Em, Hs, n), Ep, n)

    def _solve_amplitudes(self, ranks):
        n = self.order
        secN = self.secN
        self.amp_ops = {}   # k -> list of (ops, t)
        self.amps = {}
        exc = {r: self._excitations(r) for r in ranks}
        AN = [None]
        for k in range(1, n + 1):
            Aser = AN + [None]
            R = self._Ht(Aser, self.H0N, self.HN, k)[k]
            Rphi = R @ self.phi
            lst = []
            t1 = np.zeros((self.m, self.m))
            t2 = {}
            for r in ranks:
                # singles through order n, doubles (and higher) through order n-1
                if (r == 1 and k > n) or (r >= 2 and k > n - 1):
                    continue
                for (I, A, ops, D) in exc[r]:
                    vec = op_matrix(ops, secN, secN) @ self.phi
                    t = -float(vec @ Rphi) / D
                    lst.append((ops, t))
                    if r == 1:
                        t1[I[0], A[0]] = t
                    elif r == 2:
                        t2[(I[0], I[1], A[0], A[1])] = t
            self.amp_ops[k] = lst
            self.amps[k] = {"t1": t1, "t2": t2}
            AN.append(self._A_matrix(lst, secN))
        self.AN = AN
        self.AX = [None] + [self._A_matrix(self.amp_ops[k], self.secX)
                            for k in range(1, n + 1)]

    def _basis(self):
        """ADC basis h_nu^+ |Phi> as columns in the N+-1 sector, with labels."""
        cols, labels, cls = [], [], []
        if self.kind == "ea":
            for a in self.vir:
                cols.append([(a, 1)]); labels.append(("1", a)); cls.append(0)
            for i in self.occ:
                for a, b in combinations(self.vir, 2):
                    cols.append([(b, 1), (a, 1), (i, 0)])
                    labels.append(("2", (a, b, i))); cls.append(1)
        else:
            for i in self.occ:
                cols.append([(i, 0)]); labels.append(("1", i)); cls.append(0)
            for a in self.vir:
                for i, j in combinations(self.occ, 2):
                    cols.append([(a, 1), (j, 0), (i, 0)])
                    labels.append(("2", (i, j, a))); cls.append(1)
        C = np.zeros((self.secX.dim, len(cols)))
        for c, ops in enumerate(cols):
            C[:, c] = op_matrix(ops, self.secN, self.secX) @ self.phi
        return C, labels, np.array(cls)

    def _build_matrices(self):
        n = self.order
        AserN = self.AN
        AserX = self.AX
        HtN = self._Ht(AserN, self.H0N, self.HN, n)
        HtX = self._Ht(AserX, self.H0X, self.HX, n)
        dN, dX = self.secN.dim, self.secX.dim
        self.E0 = [float(self.phi @ _coef(HtN, k, dN) @ self.phi) for k in range(n + 1)]
        C, labels, cls = self._basis()
        self.labels, self.cls = labels, cls
        dim = C.shape[1]
        M = np.zeros((dim, dim))
        for k in range(n + 1):
            Mk = C.T @ _coef(HtX, k, dX) @ C - self.E0[k] * np.eye(dim)
            # a contribution of order k + class(mu) + class(nu) enters when <= n
            mask = (k + cls[:, None] + cls[None, :]) <= n
            M += np.where(mask, Mk, 0.0)
        self.M_raw = M
        self.M = M if self.kind == "ea" else M  # K = <Psi|Ht|Psi> - E0 = -M_-
        # transition moments: at_p = exp(-A) a_p exp(A)
        EpX = s_exp(AserX, n, dX)
        EmN = s_exp([None if a is None else -a for a in AserN], n, dN)
        EpN = s_exp(AserN, n, dN)
        EmX = s_exp([None if a is None else -a for a in AserX], n, dX)
        T = np.zeros((self.m, dim))
        for p in range(self.m):
            if self.kind == "ea":
                ap = op_matrix([(p, 0)], self.secX, self.secN)      # N+1 -> N
                at = s_mul(s_mul(EmN, [ap], n), EpX, n)           # N+1 -> N
                for k in range(n + 1):
                    if at[k] is None:
                        continue
                    row = self.phi @ at[k] @ C
                    T[p] += np.where(k + cls <= n, row, 0.0)
            else:
                ap = op_matrix([(p, 0)], self.secN, self.secX)      # N -> N-1
                at = s_mul(s_mul(EmX, [ap], n), EpN, n)           # N -> N-1
                for k in range(n + 1):
                    if at[k] is None:
                        continue
                    row = C.T @ (at[k] @ self.phi)
                    T[p] += np.where(k + cls <= n, row, 0.0)
        self.T = T

    # ------------------------------------------------------------------
    def exact_energies(self):
        """Full-CI ground state of N and all states of the N+-1 sector."""
        eN = np.linalg.eigvalsh(self.HN)
        eX, vX = np.linalg.eigh(self.HX)
        return eN, eX, vX

"""Unrestricted (open-shell) EA/IP-ADC(2) on the CPU in FP64, in spin orbitals
(the oracle of the unrestricted path).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.  It
shares no code with the HIP path.

The paper's unrestricted code (UADC, Sec. II and the open-shell TEMPO
calculations of Sec. V.B) works with an unrestricted Hartree-Fock reference:
alpha and beta orbitals with their own energies and their own
density-fitting factors, (p q | r s)_{st} = sum_Q B_s^Q_pq B_t^Q_rs (Eq. 38 for
each pair of spins).  This module evaluates second-order EA/IP-ADC in
spin orbitals with antisymmetrised integrals
<PQ||RS> = sum_Q (b^Q_PR b^Q_QS - b^Q_PS b^Q_QR), where b^Q_PR is B_s^Q_pr when
P and R both have spin s and 0 otherwise.  Spin orbitals are ordered alpha
first: occupied I = (alpha occ..., beta occ...), virtual A = (alpha vir...,
beta vir...).

Working equations (from Eqs. 7-14 at n = 2: M11 through second order, the
coupling at first order, the 2p1h/2h1p block at zeroth order; T, Eqs. 8/10,
with the same bookkeeping; checked term by term against the Fock-space
construction of oracle/fockspace.py, which uses no derived equation):
  t_IJ^AB = <IJ||AB> / (e_I + e_J - e_A - e_B)               (first-order doubles)
  t_I^A   = [-1/2 sum_JBC <AJ||BC> t_IJ^BC
             + 1/2 sum_JKB <JK||IB> t_JK^AB] / (e_I - e_A)     (second-order singles)
  EA (basis a_A^+|Phi>, a_C^+ a_B^+ a_I|Phi> with B < C):
    M_AB       = e_A d_AB - 1/4 sum_KLC (t_KL^AC <KL||BC> + t_KL^BC <KL||AC>)
    M_A,IBC    = -<BC||AI>
    M_IBC,IBC  = e_B + e_C - e_I
    T_pA       = d_pA - 1/4 sum_KLC t_KL^pC t_KL^AC  (p virtual);  t_p^A (p occupied)
    T_p,IBC    = -t_Ip^BC (p occupied; 0 for p virtual)
  IP (K = -M_-, basis a_I|Phi>, a_A^+ a_K a_J|Phi> with J < K):
    K_IJ       = -e_I d_IJ - 1/4 sum_KCD (t_IK^CD <JK||CD> + t_JK^CD <IK||CD>)
    K_I,JKA    = -<JK||IA>
    K_JKA,JKA  = e_A - e_J - e_K
    T_pI       = d_pI - 1/4 sum_KCD t_pK^CD t_IK^CD  (p occupied);  -t_I^p (p virtual)
    T_p,JKA    = -t_JK^Ap (p virtual; 0 for p occupied)
Spectroscopic factors P = sum_p |X_p|^2 over spin orbitals (Eq. 17), X = T Y
(Eq. 16).

Vector layout at the library boundary (both spin sectors in one vector; the
matrix is block diagonal in them):
  EA: Y1 alpha [Va], Y1 beta [Vb], then the 2p1h blocks named by the spins of
      (i, a, b): aaa [Oa][a<b packed], bab [Ob][Va][Vb] (i beta, a alpha,
      b beta), aab [Oa][Va][Vb], bbb [Ob][a<b packed]; the attached alpha
      electron's sector is (Y1 alpha, aaa, bab), the beta one's (Y1 beta,
      aab, bbb).
  IP: Y1 alpha [Oa], Y1 beta [Ob], then the 2h1p blocks named by the spins of
      (a, i, j): aaa [Va][i<j packed], bab [Vb][Oa][Ob] (a beta, i alpha,
      j beta), aab [Va][Oa][Ob], bbb [Vb][i<j packed]; removed alpha:
      (Y1 alpha, aaa, bab), removed beta: (Y1 beta, aab, bbb).
  Packed pairs p < q are ordered row-major (p, then q > p).
  A basis element is the spin-orbital state above with its two like
  indices in alpha-first order (in the mixed blocks the alpha index first).
"""
from __future__ import annotations

import numpy as np


def pairs(n):
    """Row-major list of (p, q), p < q < n."""
    return [(p, q) for p in range(n) for q in range(p + 1, n)]


class UADC2:
    """CPU FP64 unrestricted EA/IP-ADC(2)."""

    def __init__(self, eps_a, eps_b, B_a, B_b, nocc_a, nocc_b, kind):
        if kind not in ("ea", "ip"):
            raise ValueError("kind must be 'ea' or 'ip'")
        self.kind = kind
        ea, eb = np.asarray(eps_a, dtype=np.float64), np.asarray(eps_b, dtype=np.float64)
        Ba, Bb = np.asarray(B_a, dtype=np.float64), np.asarray(B_b, dtype=np.float64)
        N = ea.size
        self.N = N
        self.Oa, self.Ob = Oa, Ob = nocc_a, nocc_b
        self.Va, self.Vb = Va, Vb = N - nocc_a, N - nocc_b
        self.no, self.nv = no, nv = Oa + Ob, Va + Vb
        self.eo = np.concatenate([ea[:Oa], eb[:Ob]])
        self.ev = np.concatenate([ea[Oa:], eb[Ob:]])
        # spatial orbital of each spin orbital and its spin
        self.o_sp = np.concatenate([np.arange(Oa), np.arange(Ob)])
        self.v_sp = np.concatenate([np.arange(Oa, N), np.arange(Ob, N)])
        self.o_s = np.array([0] * Oa + [1] * Ob)
        self.v_s = np.array([0] * Va + [1] * Vb)
        B = (Ba, Bb)

        def blk(pos_p, spin_p, pos_q, spin_q):
            Q = Ba.shape[0]
            out = np.zeros((Q, len(pos_p), len(pos_q)))
            for s in range(2):
                ip = np.nonzero(spin_p == s)[0]
                iq = np.nonzero(spin_q == s)[0]
                out[np.ix_(np.arange(Q), ip, iq)] = B[s][:, pos_p[ip]][:, :, pos_q[iq]]
            return out

        self.boo = blk(self.o_sp, self.o_s, self.o_sp, self.o_s)
        self.bov = blk(self.o_sp, self.o_s, self.v_sp, self.v_s)
        self.bvv = blk(self.v_sp, self.v_s, self.v_sp, self.v_s)
        self.bvo = self.bov.transpose(0, 2, 1)
        # antisymmetrised integrals <PQ||RS> = sum_Q (b_PR b_QS - b_PS b_QR)
        d = np.einsum("Xia,Xjb->ijab", self.bov, self.bov)
        oovv = d - d.transpose(0, 1, 3, 2)                        # <IJ||AB>
        d = np.einsum("Xab,Xjc->ajbc", self.bvv, self.bov)
        vovv = d - d.transpose(0, 1, 3, 2)                        # <AJ||BC>
        ooov = (np.einsum("Xji,Xkb->jkib", self.boo, self.bov)
                - np.einsum("Xjb,Xki->jkib", self.bov, self.boo))  # <JK||IB>
        D2 = (self.eo[:, None, None, None] + self.eo[None, :, None, None]
              - self.ev[None, None, :, None] - self.ev[None, None, None, :])
        self.t = oovv / D2
        self.oovv = oovv
        D1 = self.eo[:, None] - self.ev[None, :]
        self.t1 = (-0.5 * np.einsum("ajbc,ijbc->ia", vovv, self.t)
                   + 0.5 * np.einsum("jkib,jkab->ia", ooov, self.t)) / D1
        if kind == "ea":
            tau = np.einsum("klac,klbc->ab", self.t, oovv)
            self.M11 = np.diag(self.ev) - 0.25 * (tau + tau.T)
            # C[A, I, B, C] = -<BC||AI> = -(b_BA b_CI - b_BI b_CA)
            self.C = -np.einsum("Qba,Qci->aibc", self.bvv, self.bvo) \
                + np.einsum("Qbi,Qca->aibc", self.bvo, self.bvv)
            self.rho = np.einsum("klac,klbc->ab", self.t, self.t)
        else:
            tau = np.einsum("ikcd,jkcd->ij", self.t, oovv)
            self.M11 = -np.diag(self.eo) - 0.25 * (tau + tau.T)
            # C[I, J, K, A] = -<JK||IA> = -(b_JI b_KA - b_JA b_KI)
            self.C = -np.einsum("Qji,Qka->ijka", self.boo, self.bov) \
                + np.einsum("Qja,Qki->ijka", self.bov, self.boo)
            self.rho = np.einsum("ikcd,jkcd->ij", self.t, self.t)
        self._layout()

    # ------------------------------------------------------------------
    # boundary layout <-> spin-orbital tensors
    # ------------------------------------------------------------------
    def _layout(self):
        """Spin-orbital (x, p, q) of every 2p1h/2h1p element in boundary order:
        EA (I, B, C) with B < C; IP (A, J, K) with J < K."""
        Oa, Ob, Va, Vb = self.Oa, self.Ob, self.Va, self.Vb
        idx = []
        if self.kind == "ea":
            for i in range(Oa):
                idx += [(i, a, b) for (a, b) in pairs(Va)]
            for i in range(Ob):
                idx += [(Oa + i, a, Va + b) for a in range(Va) for b in range(Vb)]
            for i in range(Oa):
                idx += [(i, a, Va + b) for a in range(Va) for b in range(Vb)]
            for i in range(Ob):
                idx += [(Oa + i, Va + a, Va + b) for (a, b) in pairs(Vb)]
            self.n1 = Va + Vb
        else:
            for a in range(Va):
                idx += [(a, i, j) for (i, j) in pairs(Oa)]
            for a in range(Vb):
                idx += [(Va + a, i, Oa + j) for i in range(Oa) for j in range(Ob)]
            for a in range(Va):
                idx += [(a, i, Oa + j) for i in range(Oa) for j in range(Ob)]
            for a in range(Vb):
                idx += [(Va + a, Oa + i, Oa + j) for (i, j) in pairs(Ob)]
            self.n1 = Oa + Ob
        self.idx2 = np.array(idx, dtype=np.int64).reshape(-1, 3)
        self.dim = self.n1 + len(idx)
        self.full_shape = (self.no, self.nv, self.nv) if self.kind == "ea" else \
            (self.nv, self.no, self.no)

    def unpack(self, vecs):
        """Y1 [z][n1] and the antisymmetric full tensor Y2 [z][...] (zero on
        spin combinations outside both sectors)."""
        vecs = np.atleast_2d(np.asarray(vecs, dtype=np.float64))
        z = vecs.shape[0]
        Y1 = vecs[:, :self.n1]
        Y2 = np.zeros((z,) + self.full_shape)
        x, p, q = self.idx2.T
        Y2[:, x, p, q] = vecs[:, self.n1:]
        Y2[:, x, q, p] = -vecs[:, self.n1:]
        return Y1, Y2

    def pack(self, S1, S2):
        x, p, q = self.idx2.T
        return np.concatenate([S1, S2[:, x, p, q]], axis=1)

    # ------------------------------------------------------------------
    # sigma, diagonal, explicit matrix
    # ------------------------------------------------------------------
    def sigma(self, vecs):
        """sigma = M Y (EA) or K Y (IP) for Y [nvec, dim] in the boundary layout."""
        Y1, Y2 = self.unpack(vecs)
        if self.kind == "ea":
            S1 = Y1 @ self.M11.T + 0.5 * np.einsum("aibc,zibc->za", self.C, Y2)
            S2 = np.einsum("aibc,za->zibc", self.C, Y1)
            d = self.ev[None, :, None] + self.ev[None, None, :] - self.eo[:, None, None]
        else:
            S1 = Y1 @ self.M11.T + 0.5 * np.einsum("ijka,zajk->zi", self.C, Y2)
            S2 = np.einsum("ijka,zi->zajk", self.C, Y1)
            d = self.ev[:, None, None] - self.eo[None, :, None] - self.eo[None, None, :]
        S2 = S2 + d[None] * Y2
        return self.pack(S1, S2)

    def diag(self):
        x, p, q = self.idx2.T
        if self.kind == "ea":
            d2 = self.ev[p] + self.ev[q] - self.eo[x]
        else:
            d2 = self.ev[x] - self.eo[p] - self.eo[q]
        return np.concatenate([np.diag(self.M11), d2])

    def explicit(self):
        return self.sigma(np.eye(self.dim)).T

    # ------------------------------------------------------------------
    # spectroscopic amplitudes and factors (Eqs. 16, 50)
    # ------------------------------------------------------------------
    def spec_amplitudes(self, vecs):
        """X [nvec][2N]: alpha orbitals 0..N-1 then beta orbitals 0..N-1."""
        Y1, Y2 = self.unpack(vecs)
        z = Y1.shape[0]
        if self.kind == "ea":
            Xv = Y1 - 0.25 * Y1 @ self.rho.T
            Xo = Y1 @ self.t1.T - 0.5 * np.einsum("ikab,ziab->zk", self.t, Y2)
        else:
            Xo = Y1 - 0.25 * Y1 @ self.rho.T
            Xv = -Y1 @ self.t1 - 0.5 * np.einsum("jkbp,zbjk->zp", self.t, Y2)
        X = np.zeros((z, 2 * self.N))
        X[:, self.o_s * self.N + self.o_sp] = Xo
        X[:, self.v_s * self.N + self.v_sp] = Xv
        return X

    def spec_factors(self, vecs):
        return np.sum(self.spec_amplitudes(vecs) ** 2, axis=1)

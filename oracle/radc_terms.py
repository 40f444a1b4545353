"""Spin-adapted (closed-shell) EA/IP-ADC(n) working equations as term tables.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle).

The paper gives no working equations (Sec. II defers them to its Ref. on the
spin-orbital derivation).  These tables were obtained from the definitions
(Eqs. 7-14) by expanding the effective Hamiltonian with the BCH series
(Eq. 11), normal ordering with respect to the reference determinant,
evaluating the matrix elements of Eqs. 7/9 and 8/10 with the order bookkeeping
described in the Fock-space module, and integrating over spin with the rules
of Eqs. 28-35.  They are checked against the Fock-space construction, which
needs no derived equation, in the test suite.

Conventions (all indices spatial):
  occupied letters i j k l m n o, virtual letters a b c d e f g h;
  g:pqrs = (pq|rs) (chemists' notation; here sum_Q B^Q_pq B^Q_rs, Eq. 38);
  f:pq   = Fock matrix = diag(eps);
  t:ijab = first-order doubles t_ij^ab = (ia|jb)/(e_i + e_j - e_a - e_b);
  u:ijab = second-order doubles; s:ia = second-order singles;
  w:ia   = third-order singles; Du, Ds = u, s times their denominators
           (e_a + e_b - e_i - e_j) and (e_a - e_i).
Vectors (the representation of Eqs. 36-37 written for this code):
  EA (an alpha electron attached):  Y1:a  and  Y2:abi, where a is the
     attached alpha particle and (b, i) a spin-conserving particle-hole pair;
     spin-orbital amplitudes Y(A,B,I) = d(sA,a)d(sB,sI) Y2:abi
                                       - d(sB,a)d(sA,sI) Y2:bai.
  IP (an alpha electron removed):   Y1:i  and  Y2:ija, where i is the removed
     alpha hole and (j, a) a spin-conserving hole-particle pair;
     Y(I,J,A) = d(sI,a)d(sJ,sA) Y2:ija - d(sJ,a)d(sI,sA) Y2:jia.
Keys "blk/k": blk is 11, 12, 21 or 22 (1 = 1p/1h, 2 = 2p1h/2h1p) and k the
order of the effective Hamiltonian; a block of ADC(n) sums k <= n - (number of
2's in blk).  Each entry is (coefficient, product of tensors); the value of a
sigma row is the sum over all indices that are not external (EA rows: a, or
a b i; IP rows: i, or i j a).  "X_p_o/k" and "X_p_v/k" give the spectroscopic
amplitude X_p (p occupied / virtual) from the at_p of order k, with the 1p/1h
part of the vector taken when k <= n and the 2p1h/2h1p part when k <= n-1.
The IP matrix is the negative of Eq. 9's (its eigenvalues are the ionisation
energies).  AMP_TERMS give the residual <Phi_mu|R^(k)|Phi> with the amplitude
of the same order left out; the amplitude is -residual/denominator (Eqs. 13-14).
"""

EA_TERMS = {
    '11/0': [
        (    '1', 'Y1:b f:ab'),
    ],
    '11/2': [
        (  '1/2', 'Y1:b t:jkca g:kcjb'),
        (   '-1', 'Y1:b t:jkca g:kbjc'),
        (  '1/2', 'Y1:b t:jkcb g:ckaj'),
        (   '-1', 'Y1:b t:jkcb g:cjak'),
    ],
    '11/3': [
        (  '1/2', 'Y1:b u:jkca g:kcjb'),
        (   '-1', 'Y1:b u:jkca g:kbjc'),
        (    '4', 'Y1:b s:jc g:jcab'),
        (   '-1', 'Y1:b s:jc g:jbac'),
        (   '-1', 'Y1:b s:jc g:cbaj'),
        (  '1/2', 'Y1:b u:jkcb g:ckaj'),
        (   '-1', 'Y1:b u:jkcb g:cjak'),
        (  '1/2', 'Du:jkbc Y1:c t:kjba'),
        (   '-1', 'Du:jkbc Y1:c t:kjab'),
        (  '1/2', 'Du:jkba Y1:c t:kjbc'),
        (   '-1', 'Du:jkba Y1:c t:kjcb'),
        (   '-2', 'Y1:b t:jkcb t:lmca g:mklj'),
        (    '1', 'Y1:b t:jkcb t:lmca g:mjlk'),
        (   '-1', 'Y1:b t:jkcb t:ljcd g:lkad'),
        (    '2', 'Y1:b t:jkcb t:ljcd g:ldak'),
        (    '2', 'Y1:b t:jkcb t:ljdc g:lkad'),
        (   '-4', 'Y1:b t:jkcb t:ljdc g:ldak'),
        (    '2', 'Y1:b t:jkbc t:ljcd g:lkad'),
        (   '-1', 'Y1:b t:jkbc t:ljcd g:ldak'),
        (   '-1', 'Y1:b t:jkbc t:ljdc g:lkad'),
        (    '2', 'Y1:b t:jkbc t:ljdc g:ldak'),
        (   '-4', 'Y1:b t:jkcd t:ljdc g:lkab'),
        (    '2', 'Y1:b t:jkcd t:ljdc g:lbak'),
        (    '2', 'Y1:b t:jkcd t:ljcd g:lkab'),
        (   '-1', 'Y1:b t:jkcd t:ljcd g:lbak'),
        (   '-1', 'Y1:b t:jkcb t:ljda g:lkcd'),
        (    '2', 'Y1:b t:jkcb t:ljda g:ldck'),
        (    '2', 'Y1:b t:jkcb t:ljad g:lkcd'),
        (   '-1', 'Y1:b t:jkcb t:ljad g:ldck'),
        (    '2', 'Y1:b t:jkbc t:ljda g:lkcd'),
        (   '-4', 'Y1:b t:jkbc t:ljda g:ldck'),
        (   '-1', 'Y1:b t:jkbc t:ljad g:lkcd'),
        (    '2', 'Y1:b t:jkbc t:ljad g:ldck'),
        (    '2', 'Y1:b t:jkcd t:ljda g:lkcb'),
        (   '-1', 'Y1:b t:jkcd t:ljda g:lbck'),
        (   '-1', 'Y1:b t:jkcd t:ljad g:lkcb'),
        (    '2', 'Y1:b t:jkcd t:ljad g:lbck'),
        (   '-1', 'Y1:b t:jkcd t:ljca g:lkdb'),
        (    '2', 'Y1:b t:jkcd t:ljca g:lbdk'),
        (    '2', 'Y1:b t:jkcd t:ljac g:lkdb'),
        (   '-4', 'Y1:b t:jkcd t:ljac g:lbdk'),
        (   '-2', 'Y1:b t:jkcb t:kjde g:cead'),
        (    '1', 'Y1:b t:jkcb t:kjde g:cdae'),
        (    '4', 'Y1:b t:jkcd t:kjde g:ceab'),
        (   '-2', 'Y1:b t:jkcd t:kjde g:cbae'),
        (   '-2', 'Y1:b t:jkcd t:kjed g:ceab'),
        (    '1', 'Y1:b t:jkcd t:kjed g:cbae'),
        (   '-2', 'Y1:b t:jkcd t:kjea g:decb'),
        (    '1', 'Y1:b t:jkcd t:kjea g:dbce'),
    ],
    '12/1': [
        (    '1', 'Y2:bcj g:jbac'),
        (   '-2', 'Y2:bcj g:jcab'),
    ],
    '12/2': [
        (   '-2', 'Y2:bcj t:klbc g:jlak'),
        (    '1', 'Y2:bcj t:klbc g:jkal'),
        (   '-2', 'Y2:baj t:klcb g:jlck'),
        (    '1', 'Y2:baj t:klcb g:jkcl'),
        (    '4', 'Y2:abj t:klcb g:jlck'),
        (   '-2', 'Y2:abj t:klcb g:jkcl'),
        (    '2', 'Y2:bcj t:jkdc g:dkab'),
        (   '-1', 'Y2:bcj t:jkdc g:dbak'),
        (   '-4', 'Y2:bcj t:jkcd g:dkab'),
        (    '2', 'Y2:bcj t:jkcd g:dbak'),
        (   '-1', 'Y2:bcj t:jkdb g:dkac'),
        (    '2', 'Y2:bcj t:jkdb g:dcak'),
        (    '2', 'Y2:bcj t:jkbd g:dkac'),
        (   '-1', 'Y2:bcj t:jkbd g:dcak'),
        (    '2', 'Y2:baj t:jkcd g:dkcb'),
        (   '-1', 'Y2:baj t:jkcd g:dbck'),
        (   '-4', 'Y2:abj t:jkcd g:dkcb'),
        (    '2', 'Y2:abj t:jkcd g:dbck'),
        (    '1', 'Ds:jb Y2:baj'),
        (   '-2', 'Ds:jb Y2:abj'),
    ],
    '21/1': [
        (   '-1', 'Y1:c g:acbi'),
    ],
    '21/2': [
        (   '-1', 'Y1:c t:jkab g:kijc'),
        (    '2', 'Y1:a t:jkcb g:kijc'),
        (   '-1', 'Y1:a t:jkcb g:kcji'),
        (    '1', 'Y1:c t:ijdb g:jdac'),
        (   '-2', 'Y1:c t:ijbd g:jdac'),
        (    '1', 'Y1:c t:ijbd g:jcad'),
        (    '1', 'Y1:c t:ijda g:jcbd'),
        (   '-2', 'Y1:a t:ijcd g:jdbc'),
        (    '1', 'Y1:a t:ijcd g:jcbd'),
        (   '-1', 'Ds:ib Y1:a'),
    ],
    '22/0': [
        (   '-1', 'Y2:abj f:ji'),
        (    '1', 'Y2:aci f:bc'),
        (    '1', 'Y2:cbi f:ac'),
    ],
    '22/1': [
        (   '-1', 'Y2:caj g:jcbi'),
        (   '-1', 'Y2:acj g:jibc'),
        (    '2', 'Y2:acj g:jcbi'),
        (   '-1', 'Y2:cbj g:jiac'),
        (    '1', 'Y2:cdi g:acbd'),
    ],
    'X_p_o/1': [
        (   '-1', 'Y2:bcj t:jpbc'),
        (    '2', 'Y2:bcj t:jpcb'),
    ],
    'X_p_o/2': [
        (   '-1', 'Y1:b s:pb'),
        (   '-1', 'Y2:bcj u:jpbc'),
        (    '2', 'Y2:bcj u:jpcb'),
    ],
    'X_p_o/3': [
        (   '-1', 'Y1:b w:pb'),
        (   '-1', 'Y1:b s:jc t:jpcb'),
        (  '1/2', 'Y1:b s:jc t:jpbc'),
    ],
    'X_p_v/0': [
        (    '1', 'Y1:p'),
    ],
    'X_p_v/2': [
        (   '-1', 'Y1:b t:jkcb t:kjpc'),
        (  '1/2', 'Y1:b t:jkcb t:kjcp'),
    ],
    'X_p_v/3': [
        (   '-1', 'Y1:b t:jkpc u:kjcb'),
        (  '1/2', 'Y1:b t:jkpc u:kjbc'),
        (   '-1', 'Y1:b t:jkcb u:kjpc'),
        (  '1/2', 'Y1:b t:jkcb u:kjcp'),
    ],
}

IP_TERMS = {
    '11/0': [
        (   '-1', 'Y1:j f:ji'),
    ],
    '11/2': [
        (  '1/2', 'Y1:j t:ikbc g:jckb'),
        (   '-1', 'Y1:j t:ikbc g:jbkc'),
        (  '1/2', 'Y1:j t:jkbc g:cibk'),
        (   '-1', 'Y1:j t:jkbc g:ckbi'),
    ],
    '11/3': [
        (   '-4', 'Y1:j s:kb g:jikb'),
        (    '1', 'Y1:j s:kb g:jbki'),
        (  '1/2', 'Y1:j u:ikbc g:jckb'),
        (   '-1', 'Y1:j u:ikbc g:jbkc'),
        (    '1', 'Y1:j s:kb g:jkbi'),
        (  '1/2', 'Y1:j u:jkbc g:cibk'),
        (   '-1', 'Y1:j u:jkbc g:ckbi'),
        (  '1/2', 'Du:jkbc Y1:j t:ikcb'),
        (   '-1', 'Du:jkbc Y1:j t:ikbc'),
        (  '1/2', 'Du:ijbc Y1:k t:kjcb'),
        (   '-1', 'Du:ijbc Y1:k t:kjbc'),
        (   '-2', 'Y1:j t:jkbc t:lmcb g:milk'),
        (    '1', 'Y1:j t:jkbc t:lmcb g:mkli'),
        (    '4', 'Y1:j t:klbc t:mkcb g:jiml'),
        (   '-2', 'Y1:j t:klbc t:mkcb g:jlmi'),
        (   '-2', 'Y1:j t:klbc t:mkbc g:jiml'),
        (    '1', 'Y1:j t:klbc t:mkbc g:jlmi'),
        (   '-2', 'Y1:j t:ikbc t:lmcb g:jmkl'),
        (    '1', 'Y1:j t:ikbc t:lmcb g:jlkm'),
        (   '-1', 'Y1:j t:jkbc t:lkcd g:libd'),
        (    '2', 'Y1:j t:jkbc t:lkcd g:ldbi'),
        (    '2', 'Y1:j t:jkbc t:lkdc g:libd'),
        (   '-4', 'Y1:j t:jkbc t:lkdc g:ldbi'),
        (    '2', 'Y1:j t:jkbc t:lkbd g:licd'),
        (   '-1', 'Y1:j t:jkbc t:lkbd g:ldci'),
        (   '-1', 'Y1:j t:jkbc t:lkdb g:licd'),
        (    '2', 'Y1:j t:jkbc t:lkdb g:ldci'),
        (   '-4', 'Y1:j t:klbc t:lkcd g:jibd'),
        (    '2', 'Y1:j t:klbc t:lkcd g:jdbi'),
        (    '2', 'Y1:j t:klbc t:lkdc g:jibd'),
        (   '-1', 'Y1:j t:klbc t:lkdc g:jdbi'),
        (   '-1', 'Y1:j t:ikbc t:jldb g:kldc'),
        (    '2', 'Y1:j t:ikbc t:jldb g:kcdl'),
        (    '2', 'Y1:j t:ikbc t:jlbd g:kldc'),
        (   '-4', 'Y1:j t:ikbc t:jlbd g:kcdl'),
        (    '2', 'Y1:j t:ikbc t:jldc g:kldb'),
        (   '-1', 'Y1:j t:ikbc t:jldc g:kbdl'),
        (   '-1', 'Y1:j t:ikbc t:jlcd g:kldb'),
        (    '2', 'Y1:j t:ikbc t:jlcd g:kbdl'),
        (    '2', 'Y1:j t:ikbc t:kldb g:jldc'),
        (   '-1', 'Y1:j t:ikbc t:kldb g:jcdl'),
        (   '-1', 'Y1:j t:ikbc t:klbd g:jldc'),
        (    '2', 'Y1:j t:ikbc t:klbd g:jcdl'),
        (   '-1', 'Y1:j t:ikbc t:kldc g:jldb'),
        (    '2', 'Y1:j t:ikbc t:kldc g:jbdl'),
        (    '2', 'Y1:j t:ikbc t:klcd g:jldb'),
        (   '-4', 'Y1:j t:ikbc t:klcd g:jbdl'),
        (   '-2', 'Y1:j t:ikbc t:jkde g:ecdb'),
        (    '1', 'Y1:j t:ikbc t:jkde g:ebdc'),
    ],
    '12/1': [
        (    '1', 'Y2:jkb g:kijb'),
        (   '-2', 'Y2:jkb g:kbji'),
    ],
    '12/2': [
        (    '2', 'Y2:jkb t:klcb g:jicl'),
        (   '-1', 'Y2:jkb t:klcb g:jlci'),
        (   '-4', 'Y2:jkb t:klbc g:jicl'),
        (    '2', 'Y2:jkb t:klbc g:jlci'),
        (   '-1', 'Y2:jkb t:jlcb g:kicl'),
        (    '2', 'Y2:jkb t:jlcb g:klci'),
        (    '2', 'Y2:jkb t:jlbc g:kicl'),
        (   '-1', 'Y2:jkb t:jlbc g:klci'),
        (    '2', 'Y2:jib t:klcb g:jlck'),
        (   '-1', 'Y2:jib t:klcb g:jkcl'),
        (   '-4', 'Y2:ijb t:klcb g:jlck'),
        (    '2', 'Y2:ijb t:klcb g:jkcl'),
        (   '-2', 'Y2:jkb t:kjcd g:dicb'),
        (    '1', 'Y2:jkb t:kjcd g:dbci'),
        (   '-2', 'Y2:jib t:jkcd g:dkcb'),
        (    '1', 'Y2:jib t:jkcd g:dbck'),
        (    '4', 'Y2:ijb t:jkcd g:dkcb'),
        (   '-2', 'Y2:ijb t:jkcd g:dbck'),
        (   '-1', 'Ds:jb Y2:jib'),
        (    '2', 'Ds:jb Y2:ijb'),
    ],
    '21/1': [
        (   '-1', 'Y1:k g:kiaj'),
    ],
    '21/2': [
        (    '1', 'Y1:k t:jlba g:kilb'),
        (   '-2', 'Y1:k t:jlab g:kilb'),
        (    '1', 'Y1:k t:jlab g:kbli'),
        (    '1', 'Y1:k t:ilba g:kblj'),
        (   '-2', 'Y1:i t:klba g:ljkb'),
        (    '1', 'Y1:i t:klba g:lbkj'),
        (   '-1', 'Y1:k t:jibc g:kcab'),
        (    '2', 'Y1:i t:jkbc g:kcab'),
        (   '-1', 'Y1:i t:jkbc g:kbac'),
        (    '1', 'Ds:ja Y1:i'),
    ],
    '22/0': [
        (   '-1', 'Y2:ika f:kj'),
        (   '-1', 'Y2:kja f:ki'),
        (    '1', 'Y2:ijb f:ab'),
    ],
    '22/1': [
        (    '1', 'Y2:kla g:ljki'),
        (   '-1', 'Y2:kib g:kbaj'),
        (   '-1', 'Y2:ikb g:kjab'),
        (    '2', 'Y2:ikb g:kbaj'),
        (   '-1', 'Y2:kjb g:kiab'),
    ],
    'X_p_o/0': [
        (    '1', 'Y1:p'),
    ],
    'X_p_o/2': [
        (   '-1', 'Y1:j t:jkbc t:kpcb'),
        (  '1/2', 'Y1:j t:jkbc t:kpbc'),
    ],
    'X_p_o/3': [
        (   '-1', 'Y1:j t:kpbc u:jkcb'),
        (  '1/2', 'Y1:j t:kpbc u:jkbc'),
        (   '-1', 'Y1:j t:jkbc u:kpcb'),
        (  '1/2', 'Y1:j t:jkbc u:kpbc'),
    ],
    'X_p_v/1': [
        (   '-1', 'Y2:jkb t:kjpb'),
        (    '2', 'Y2:jkb t:kjbp'),
    ],
    'X_p_v/2': [
        (    '1', 'Y1:j s:jp'),
        (   '-1', 'Y2:jkb u:kjpb'),
        (    '2', 'Y2:jkb u:kjbp'),
    ],
    'X_p_v/3': [
        (    '1', 'Y1:j w:jp'),
        (    '1', 'Y1:j s:kb t:jkpb'),
        ( '-1/2', 'Y1:j s:kb t:jkbp'),
    ],
}

AMP_TERMS = {
    't1_2': [
        (   '-2', 't:jkba g:kijb'),
        (    '1', 't:jkba g:kbji'),
        (    '2', 't:ijbc g:jcab'),
        (   '-1', 't:ijbc g:jbac'),
    ],
    't2_2': [
        (    '1', 't:klba g:likj'),
        (   '-1', 't:jkca g:kibc'),
        (   '-1', 't:jkcb g:kcai'),
        (   '-1', 't:jkbc g:kiac'),
        (    '2', 't:jkbc g:kcai'),
        (   '-1', 't:ikca g:kcbj'),
        (   '-1', 't:ikac g:kjbc'),
        (    '2', 't:ikac g:kcbj'),
        (   '-1', 't:ikcb g:kjac'),
        (    '1', 't:jicd g:bcad'),
    ],
    't1_3': [
        (   '-2', 'u:jkba g:kijb'),
        (    '1', 'u:jkba g:kbji'),
        (   '-1', 's:jb g:jiab'),
        (    '3', 's:jb g:jbai'),
        (    '2', 'u:ijbc g:jcab'),
        (   '-1', 'u:ijbc g:jbac'),
        ( '-1/2', 's:jb g:biaj'),
        ( '-1/2', 'Ds:jb t:ijba'),
        (    '1', 'Ds:jb t:ijab'),
        (    '2', 't:jkbc t:ljcb g:liak'),
        (   '-4', 't:jkbc t:ljcb g:lkai'),
        (   '-1', 't:jkbc t:ljbc g:liak'),
        (    '2', 't:jkbc t:ljbc g:lkai'),
        (   '-1', 't:jkbc t:ljca g:libk'),
        (    '2', 't:jkbc t:ljca g:lkbi'),
        (    '2', 't:jkbc t:ljac g:libk'),
        (   '-1', 't:jkbc t:ljac g:lkbi'),
        (    '2', 't:jkbc t:ljba g:lick'),
        (   '-1', 't:jkbc t:ljba g:lkci'),
        (   '-4', 't:jkbc t:ljab g:lick'),
        (    '2', 't:jkbc t:ljab g:lkci'),
        (   '-1', 't:ijbc t:klcb g:jlak'),
        (    '2', 't:ijbc t:klcb g:jkal'),
        (    '2', 't:ijba t:klcb g:jlck'),
        (   '-1', 't:ijba t:klcb g:jkcl'),
        (   '-4', 't:ijab t:klcb g:jlck'),
        (    '2', 't:ijab t:klcb g:jkcl'),
        (   '-2', 't:jkbc t:kjcd g:biad'),
        (    '4', 't:jkbc t:kjcd g:bdai'),
        (    '1', 't:jkbc t:kjdc g:biad'),
        (   '-2', 't:jkbc t:kjdc g:bdai'),
        (    '1', 't:jkbc t:kjda g:cibd'),
        (   '-2', 't:jkbc t:kjda g:cdbi'),
        (    '1', 't:ijbc t:jkdb g:dkac'),
        (   '-2', 't:ijbc t:jkdb g:dcak'),
        (   '-2', 't:ijbc t:jkbd g:dkac'),
        (    '1', 't:ijbc t:jkbd g:dcak'),
        (   '-2', 't:ijbc t:jkdc g:dkab'),
        (    '1', 't:ijbc t:jkdc g:dbak'),
        (    '4', 't:ijbc t:jkcd g:dkab'),
        (   '-2', 't:ijbc t:jkcd g:dbak'),
        (   '-2', 't:ijba t:jkcd g:dkcb'),
        (    '1', 't:ijba t:jkcd g:dbck'),
        (    '4', 't:ijab t:jkcd g:dkcb'),
        (   '-2', 't:ijab t:jkcd g:dbck'),
    ],
}

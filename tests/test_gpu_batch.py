"""Solves of several uneven systems together (adc_batch_davidson: lockstep, or
concurrent on host threads, each with and without sigma graphs; and the
batch object of adc_setup_batch / adc_davidson_batch) against the
single-system solver on each (same sigma kernels, same solver steps, so the
same roots and iteration counts) and against the CPU oracle's eigenpairs of
each system (oracle sigma + oracle Davidson): roots to 1e-8 Eh, Eq. 50
factors to 1e-5 of max(1, |P|)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _systems():
    """Uneven systems of the batched EA-ADC(2) family (nocc capped at 10) plus
    one EA-ADC(3) and one IP-ADC(3) system."""
    from synthetic import make_batch_system, small_system
    out = []
    for s in (0, 1, 2):
        eps, B, (O, V, Q) = make_batch_system(s, 10)
        out.append((eps, B, O, 2, "ea"))
    eps, B = small_system(4, 30, 70, 41)
    out.append((eps, B, 4, 3, "ea"))
    eps, B = small_system(6, 25, 60, 42)
    out.append((eps, B, 6, 3, "ip"))
    return out


def _contexts(systems, precision=0):
    import paper_2012_06714_amd as adc
    dev = torch.device("cuda:0")
    ctxs = []
    for eps, B, O, order, kind in systems:
        c = adc.Context(torch.tensor(eps, device=dev), torch.tensor(B, device=dev), O, order, kind)
        c.set_option("tol_e", 1e-10)
        c.set_option("tol_r", 1e-7)
        c.set_option("block", 4)
        c.set_option("precision", precision)
        ctxs.append(c)
    return ctxs


_ORACLE = {}


def _oracle_roots(systems, nroots):
    """Lowest roots and factors of each system from the oracle alone (cached)."""
    from oracle.davidson import davidson
    from oracle.radc import RADC
    if nroots not in _ORACLE:
        out = []
        for eps, B, O, order, kind in systems:
            r = RADC(eps, B, O, order, kind)
            w, v, _, conv = davidson(r.sigma, r.diag(), nroots, block=8, tol_e=1e-11,
                                     tol_r=1e-7, max_iter=400)
            assert conv
            out.append((w, r.spec_factors(v)))
        _ORACLE[nroots] = out
    return _ORACLE[nroots]


def _check_oracle(systems, e, P):
    for k, (w, Pr) in enumerate(_oracle_roots(systems, 3)):
        assert np.abs(e[k] - w).max() < 1e-8, (k, e[k], w)
        assert (np.abs(P[k] - Pr) / np.maximum(1, np.abs(Pr))).max() < 1e-5, (k, P[k], Pr)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_single_solves(precision):
    import paper_2012_06714_amd as adc
    systems = _systems()
    _say(f"case batch precision={precision}")
    ref = []
    for c in _contexts(systems, precision):
        e, P, _, it, ok = c.davidson(3, want_vectors=False)
        ref.append((np.array(e), np.array(P), it, ok))
        c.close()
    for use_graph, concurrent, threads in ((True, False, 0), (False, False, 0), (True, True, 0),
                                           (False, True, 0), (True, True, 2)):
        ctxs = _contexts(systems, precision)
        e, P, it, st, stats = adc.batch_davidson(ctxs, 3, use_graph=use_graph,
                                                 concurrent=concurrent, threads=threads)
        for c in ctxs:
            c.close()
        _say(f"graph={use_graph} concurrent={concurrent} threads={threads} stats {stats} "
             f"iterations {list(it)}")
        for k, (e0, P0, it0, ok0) in enumerate(ref):
            assert ok0 and st[k] == 0
            assert it[k] == it0
            assert np.abs(e[k] - e0).max() < 1e-10
            assert (np.abs(P[k] - P0) / np.maximum(1, np.abs(P0))).max() < 1e-9
        _check_oracle(systems, e, P)
        if use_graph:
            # one replay per active system and iteration; graphs captured per
            # (system, vector count, precision), reused across iterations
            assert stats["graph_launches"] == sum(int(i) for i in it)
            assert 1 <= stats["captures"] < stats["graph_launches"]
            if not concurrent:
                # lockstep: at most one launch of the combined graph per iteration,
                # re-instantiated only when the set of systems/vector counts changes
                assert 1 <= stats["launches"] <= stats["iterations"]
                assert 1 <= stats["instantiations"] <= stats["launches"]


def test_batch_object_matches_oracle():
    """adc_setup_batch + adc_batch_set_option + adc_davidson_batch."""
    import paper_2012_06714_amd as adc
    systems = _systems()
    _say("case batch object")
    dev = torch.device("cuda:0")
    b = adc.Batch([(torch.tensor(eps, device=dev), torch.tensor(B, device=dev), O, order, kind)
                   for eps, B, O, order, kind in systems])
    for k, v in (("tol_e", 1e-10), ("tol_r", 1e-7), ("block", 4)):
        b.set_option(k, v)
    e, P, it, st, stats = b.davidson(3, use_graph=True)
    b.close()
    assert np.all(st == 0)
    _check_oracle(systems, e, P)

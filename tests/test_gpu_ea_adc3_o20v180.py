"""The EA-ADC(3) O=20, V=180, Naux=600 workload (8 roots, block 16) solved on
the GPU against the stored reference of the CPU oracle
(tests/golden/ea_adc3_o20v180_roots.json, written by
tests/golden/make_ea_adc3_o20v180.py from oracle.radc and oracle.davidson
alone).  Bounds: eigenvalues within 1e-6 Eh, spectroscopic factors (Eq. 50)
within 1e-5 of max(1, |P|), for the FP64 solve and the mixed-precision solves
(BF16 products, then FP64 refinement; BF16 then FP32 then FP64)."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "ea_adc3_o20v180_roots.json")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2012_06714_amd as adc
    from synthetic import make_system
    eps, B, wl = make_system("c2")
    c = adc.Context(torch.tensor(eps, device="cuda"), torch.tensor(B, device="cuda"), wl.nocc,
                    wl.order, wl.kind)
    yield c
    c.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_roots_match_stored_oracle_solve(ctx, precision):
    ref = json.load(open(GOLDEN))
    assert ref["converged"]
    e_ref = np.array(ref["energies_Eh"])
    P_ref = np.array(ref["spec_factors"])
    _say(f"case ea-adc3-o20v180 precision={precision}")
    for k, v in (("precision", precision), ("block", 16), ("tol_e", 1e-8), ("tol_r", 1e-8),
                 ("max_iter", 300)):
        ctx.set_option(k, v)
    e, P, _, it, conv = ctx.davidson(len(e_ref), want_vectors=False)
    err_e = np.abs(np.array(e) - e_ref)
    err_p = np.abs(np.array(P) - P_ref) / np.maximum(1.0, np.abs(P_ref))
    _say(f"  {it} iterations, max |dE| {err_e.max():.3e} Eh, max |dP|/max(1,|P|) "
         f"{err_p.max():.3e}")
    assert conv
    assert err_e.max() <= 1e-6
    assert err_p.max() <= 1e-5

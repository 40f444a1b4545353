"""The memory-bounded paths used for the largest systems, forced on small ones
and compared with the CPU oracle:

* the setup's large contractions evaluated in slices (a tiny slice budget
  splits every four-index product into many slices and runs every blocked
  loop one occupied index at a time), with B handed over in host memory;
* the blocked EA sigma (option ea_layout = 2): the product-ready operands
  built per call, one block at a time, from t, (ov|ov) and (oo|vv), at every
  precision level; t~ + u~ parked in host memory for the spectroscopic
  amplitudes.

Bounds: FP64 sigma and diagonal to 1e-12 of the largest element (as the
plain parity test), reduced-precision sigma element by element against the
oracle's magnitude of the same sums (BF16 products 6e-3, FP32 products 1e-6),
Eq. 50 factors to 1e-10 of max(1, |P|)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sliced_ctx(eps, B, O, order, kind, budget):
    import paper_2012_06714_amd as adc
    adc.set_setup_option("slice_budget", budget)
    try:
        return adc.Context(torch.tensor(eps, device="cuda"), np.ascontiguousarray(B), O, order,
                           kind)
    finally:
        adc.set_setup_option("slice_budget", 0)


@pytest.mark.parametrize("kind,order", [("ea", 3), ("ip", 3), ("ea", 2), ("ip", 2)])
def test_sliced_setup_from_host_input_matches_oracle(kind, order):
    from oracle.radc import RADC
    from synthetic import random_vectors, small_system
    O, V, Q = 4, 11, 33
    eps, B = small_system(O, V, Q, 61)
    _say(f"case sliced setup {kind} n={order}")
    ref = RADC(eps, B, O, order, kind)
    ctx = _sliced_ctx(eps, B, O, order, kind, 200)
    X = random_vectors(ref.dim, 5, 62)
    s_ref = ref.sigma(X)
    s = ctx.sigma(torch.tensor(X, device="cuda")).cpu().numpy()
    assert np.abs(s - s_ref).max() <= 1e-12 * np.abs(s_ref).max()
    d_ref = ref.diag()
    assert np.abs(ctx.diag().cpu().numpy() - d_ref).max() <= 1e-12 * np.abs(d_ref).max()
    V0 = random_vectors(ref.dim, 3, 63)
    V0 /= np.linalg.norm(V0, axis=1, keepdims=True)
    P, _ = ctx.spec_factors(torch.tensor(V0, device="cuda"))
    P_ref = ref.spec_factors(V0)
    assert (np.abs(np.array(P) - P_ref) / np.maximum(1, np.abs(P_ref))).max() <= 1e-10
    ctx.close()


# BF16 products: every operand is rounded to 8 bits once (relative 2^-9) and a
# few intermediates once more, so an element's error stays below about
# 3 x 2^-9 of the magnitude of its products; FP32 products: sums of up to
# V^2 terms at 2^-24
LEVEL_TOL = {1: 6e-3, 2: 1e-6}


def test_blocked_ea_sigma_matches_oracle():
    from oracle.radc import RADC
    from synthetic import random_vectors, small_system
    O, V, Q = 5, 40, 90
    eps, B = small_system(O, V, Q, 64)
    _say("case blocked EA sigma")
    ref = RADC(eps, B, O, 3, "ea")
    X = random_vectors(ref.dim, 4, 65)
    s_ref = ref.sigma(X)
    mag = ref.sigma_magnitude(X)
    # blocks of one leading index in every blocked product
    ctx = _sliced_ctx(eps, B, O, 3, "ea", 100)
    ctx.set_option("ea_layout", 2)
    Xd = torch.tensor(X, device="cuda")
    for level in (0, 1, 2):
        ctx.set_option("precision", level)
        s = ctx.sigma(Xd).cpu().numpy()
        if level == 0:
            err = np.abs(s - s_ref).max() / np.abs(s_ref).max()
            _say(f"  level 0: max |err| / max |sigma| {err:.3e}")
            assert err <= 1e-12
        else:
            ratio = float((np.abs(s - s_ref) / (mag + 1e-300)).max())
            _say(f"  level {level}: max |err| / magnitude {ratio:.3e}")
            assert ratio <= LEVEL_TOL[level]
    # t~ + u~ now lives in host memory: the factors stream it back in blocks
    V0 = random_vectors(ref.dim, 3, 66)
    V0 /= np.linalg.norm(V0, axis=1, keepdims=True)
    P, Xs = ctx.spec_factors(torch.tensor(V0, device="cuda"))
    P_ref = ref.spec_factors(V0)
    assert (np.abs(np.array(P) - P_ref) / np.maximum(1, np.abs(P_ref))).max() <= 1e-10
    # a solve on the blocked path (FP64, then the mixed mode) against the oracle's
    from oracle.davidson import davidson
    w, vec, _, conv = davidson(ref.sigma, ref.diag(), 3, block=6, tol_e=1e-11, tol_r=1e-7)
    assert conv
    Pw = ref.spec_factors(vec)
    for level in (0, 1):
        ctx.set_option("precision", level)
        ctx.set_option("tol_e", 1e-10)
        ctx.set_option("tol_r", 1e-8)
        e, Pd, _, it, ok = ctx.davidson(3, want_vectors=False)
        _say(f"  solve level {level}: {it} iterations, max |dE| "
             f"{np.abs(np.array(e) - w).max():.3e}")
        assert ok
        assert np.abs(np.array(e) - w).max() < 1e-8
        assert (np.abs(np.array(Pd) - Pw) / np.maximum(1, np.abs(Pw))).max() < 1e-5
    ctx.close()


@pytest.mark.parametrize("order", [3, 2])
def test_out_of_core_bvv_matches_oracle(order):
    """Option bvv_host: B_vv and its FP32 / BF16 copies in pinned host memory,
    staged per product one block of rows at a time (a tiny slice budget makes
    every block one virtual index), with the blocked and resident EA paths;
    then moved back to the device."""
    from oracle.radc import RADC
    from synthetic import random_vectors, small_system
    O, V, Q = 4, 24, 60
    eps, B = small_system(O, V, Q, 81)
    _say(f"case out-of-core B_vv n={order}")
    ref = RADC(eps, B, O, order, "ea")
    X = random_vectors(ref.dim, 3, 82)
    s_ref = ref.sigma(X)
    mag = ref.sigma_magnitude(X)
    ctx = _sliced_ctx(eps, B, O, order, "ea", 100)
    Xd = torch.tensor(X, device="cuda")
    s_dev = ctx.sigma(Xd).cpu().numpy()
    ctx.set_option("bvv_host", 1)
    for layout in ((1, 2) if order == 3 else (1,)):
        ctx.set_option("ea_layout", layout)
        for level in (0, 1, 2):
            ctx.set_option("precision", level)
            s = ctx.sigma(Xd).cpu().numpy()
            if level == 0:
                err = np.abs(s - s_ref).max() / np.abs(s_ref).max()
                _say(f"  layout {layout} level 0: {err:.3e}")
                assert err <= 1e-12
            else:
                ratio = float((np.abs(s - s_ref) / (mag + 1e-300)).max())
                _say(f"  layout {layout} level {level}: {ratio:.3e}")
                assert ratio <= LEVEL_TOL[level]
    ctx.set_option("precision", 0)
    ctx.set_option("tol_e", 1e-10)
    ctx.set_option("tol_r", 1e-8)
    e, P, _, it, ok = ctx.davidson(3, want_vectors=False)
    assert ok
    from oracle.davidson import davidson
    w, vec, _, conv = davidson(ref.sigma, ref.diag(), 3, block=6, tol_e=1e-11, tol_r=1e-7)
    assert conv and np.abs(np.array(e) - w).max() < 1e-8
    ctx.set_option("bvv_host", 0)
    s_back = ctx.sigma(Xd).cpu().numpy()
    assert np.abs(s_back - s_dev).max() <= 1e-13 * np.abs(s_dev).max()
    ctx.close()


@pytest.mark.parametrize("kind,order", [("ea", 3), ("ip", 3), ("ea", 2), ("ip", 2)])
def test_m11_on_the_fly_matches_oracle(kind, order):
    """Setup option m11_onthefly: no precomputed 1p-1p / 1h-1h block; sigma
    applies it through intermediates every call (FP64 at every level).  Sigma
    at every precision level and the solved roots against the oracle."""
    import paper_2012_06714_amd as adc
    from oracle.radc import RADC
    from synthetic import random_vectors, small_system
    O, V, Q = 4, 13, 35
    eps, B = small_system(O, V, Q, 91)
    _say(f"case on-the-fly 11 block {kind} n={order}")
    ref = RADC(eps, B, O, order, kind)
    adc.set_setup_option("m11_onthefly", 1)
    try:
        ctx = adc.Context(torch.tensor(eps, device="cuda"), torch.tensor(B, device="cuda"), O,
                          order, kind)
    finally:
        adc.set_setup_option("m11_onthefly", 0)
    X = random_vectors(ref.dim, 4, 92)
    s_ref = ref.sigma(X)
    mag = ref.sigma_magnitude(X)
    Xd = torch.tensor(X, device="cuda")
    for level in (0, 1, 2):
        ctx.set_option("precision", level)
        s = ctx.sigma(Xd).cpu().numpy()
        if level == 0:
            err = np.abs(s - s_ref).max() / np.abs(s_ref).max()
            _say(f"  level 0: {err:.3e}")
            assert err <= 1e-12
        else:
            ratio = float((np.abs(s - s_ref) / (mag + 1e-300)).max())
            _say(f"  level {level}: {ratio:.3e}")
            assert ratio <= LEVEL_TOL[level]
    ctx.set_option("precision", 0)
    ctx.set_option("tol_e", 1e-10)
    ctx.set_option("tol_r", 1e-8)
    e, P, _, it, ok = ctx.davidson(3, want_vectors=False)
    w, v = np.linalg.eigh(ref.explicit())
    assert ok and np.abs(np.array(e) - w[:3]).max() < 1e-8
    P_ref = ref.spec_factors(v[:, :3].T)
    assert (np.abs(np.array(P) - P_ref) / np.maximum(1, np.abs(P_ref))).max() < 1e-6
    ctx.close()

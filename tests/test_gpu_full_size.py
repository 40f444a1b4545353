"""Parity at the full sizes of the workloads, where the oracle's whole sigma is
out of reach: sampled elements of the 2p1h / 2h1p rows of sigma = M_Z X,
computed one by one by the oracle (oracle.radc.RADC.sigma_rows), against the
GPU's FP64 sigma in the launch configuration the benchmark times (8 trial
vectors; the EA 1028-orbital system on the blocked path, B from host memory).

* EA-ADC(3), O=40, V=460, Naux=1400: always (about a minute);
* EA- and IP-ADC(3), O=60, V=968, Naux=3000 (1028 orbitals): only when
  ADC_FULL_SIZE=1, since their setup alone takes several minutes.

Bound: 1e-11 of the largest sampled element (FP64 sums of up to V^2 Naux
terms in different orders)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rows(nx, npair, n, seed):
    rng = np.random.default_rng(seed)
    rows = [(0, 0, 0), (nx - 1, npair - 1, npair - 1), (0, 0, npair - 1), (nx - 1, npair - 1, 0),
            (nx // 2, 3, 3)]
    while len(rows) < n:
        rows.append((int(rng.integers(nx)), int(rng.integers(npair)), int(rng.integers(npair))))
    return rows


def _check(key, nrows):
    import paper_2012_06714_amd as adc
    from oracle.radc import RADC
    from synthetic import make_system, random_vectors
    eps, B, wl = make_system(key)
    _say(f"case full-size {wl.name}: GPU setup")
    adc.set_setup_option("verbose", 1)
    try:
        ctx = adc.Context(torch.tensor(eps, device="cuda"), B, wl.nocc, wl.order, wl.kind)
    finally:
        adc.set_setup_option("verbose", 0)
    X = random_vectors(ctx.dim, 8, 5)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Y = ctx.sigma(torch.tensor(X, device="cuda")).cpu().numpy()
    nx, npair = (wl.nocc, wl.nvir) if wl.kind == "ea" else (wl.nvir, wl.nocc)
    n1 = wl.nvir if wl.kind == "ea" else wl.nocc
    ctx.close()
    del ctx
    _say(f"case full-size {wl.name}: oracle rows")
    ref = RADC(eps, B, wl.nocc, wl.order, wl.kind, lazy=True)
    del B
    rows = _rows(nx, npair, nrows, 6)
    S = ref.sigma_rows(X, rows)
    idx = [n1 + (x * npair + p) * npair + q for (x, p, q) in rows]
    got = Y[:, idx]
    err = float(np.abs(got - S).max() / np.abs(S).max())
    _say(f"  {len(rows)} rows x 8 vectors: max |GPU - oracle| / max |sigma| {err:.3e}")
    assert err <= 1e-11


def test_sampled_rows_o40v460():
    _check("c3", 40)


@pytest.mark.skipif(os.environ.get("ADC_FULL_SIZE") != "1",
                    reason="1028-orbital setup takes minutes: set ADC_FULL_SIZE=1")
@pytest.mark.parametrize("key", ["c4ea", "c4ip"])
def test_sampled_rows_1028_orbitals(key):
    _check(key, 24)

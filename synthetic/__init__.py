"""Seeded synthetic inputs for the EA/IP-ADC(n) hot path.

This module holds no ADC arithmetic.  It only draws orbital energies and
three-index density-fitting factors B^Q_pq with the distributions used for
every workload of this project (the paper's molecules, basis sets and RI fits
are not available; these synthetic systems stand in for them):

* occupied energies  ~ U[-2.0, -0.3] Eh, sorted ascending;
* virtual energies   ~ U[ 0.1,  5.0] Eh, sorted ascending;
* B^Q_pq (Q = 0 .. Naux-1, 0-based) symmetric in pq, every element, the
  diagonal included, with standard deviation 0.3*exp(-Q/40).  Per Q, in Q
  order, one call draws the packed upper triangle p <= q (row-major) from
  N(0, 1); it is scaled and mirrored.

Orbital order: occupied first, then virtual.  B is returned as a C-contiguous
float64 array of shape [Naux, N, N].  The DF factorisation
(pq|rs) ~= sum_Q B^Q_pq B^Q_rs is the approximation of the density-fitting
section (Sec. III.C, Eq. 38); B itself is taken as given.

Seeds: system s of workload c uses seed 2012067140 + 1000*c + s with numpy's
PCG64 ``default_rng``.
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np

SEED_BASE = 2012067140


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    kind: str          # "ip" or "ea"
    order: int         # ADC order, 2 or 3
    nocc: int
    nvir: int
    naux: int
    nroots: int
    block: int         # trial vectors per sigma launch
    precision: str     # "fp64" or "mixed"
    index: int         # workload number used in the seed formula


# The five workloads (sizes and solver settings).  c5 is a batch of systems
# whose sizes are themselves drawn (see draw_batch_sizes).
WORKLOADS = {
    "c1": Workload("ip-adc2-o5v19", "ip", 2, 5, 19, 72, 4, 4, "fp64", 1),
    "c2": Workload("ea-adc3-o20v180", "ea", 3, 20, 180, 600, 8, 16, "fp64", 2),
    "c3": Workload("ea-adc3-o40v460", "ea", 3, 40, 460, 1400, 16, 32, "mixed", 3),
    # 1028 orbitals: block 8 (one trial vector per root; a 16-vector BF16 sigma
    # takes about 11 s here)
    "c4ea": Workload("ea-adc3-o60v968", "ea", 3, 60, 968, 3000, 8, 8, "mixed", 4),
    "c4ip": Workload("ip-adc3-o60v968", "ip", 3, 60, 968, 3000, 8, 8, "mixed", 4),
}


def seed_for(index: int, system: int = 0) -> int:
    return SEED_BASE + 1000 * index + system


def draw_system(nocc: int, nvir: int, naux: int, seed: int,
                rng: np.random.Generator | None = None):
    """Return (eps[N], B[Naux, N, N]) drawn with the recipe above."""
    if rng is None:
        rng = np.random.default_rng(seed)
    n = nocc + nvir
    eps_o = np.sort(rng.uniform(-2.0, -0.3, size=nocc))
    eps_v = np.sort(rng.uniform(0.1, 5.0, size=nvir))
    eps = np.concatenate([eps_o, eps_v]).astype(np.float64)
    iu, ju = np.triu_indices(n)
    B = np.empty((naux, n, n), dtype=np.float64)

    def fill(q, x):
        m = B[q]
        m[iu, ju] = x
        m[ju, iu] = x

    if naux * n * n < (1 << 24):
        for q in range(naux):
            fill(q, rng.standard_normal(iu.size) * (0.3 * np.exp(-q / 40.0)))
        return eps, B
    # large systems: the draws stay in Q order on this thread (the values are
    # those of the loop above); the scatter into B runs on worker threads, at
    # most 2 per worker in flight
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(8, len(os.sched_getaffinity(0)) - 1))
    with ThreadPoolExecutor(workers) as pool:
        pending = []
        for q in range(naux):
            pending.append(pool.submit(fill, q,
                                       rng.standard_normal(iu.size) * (0.3 * np.exp(-q / 40.0))))
            if len(pending) > 2 * workers:
                pending.pop(0).result()
        for f in pending:
            f.result()
    return eps, B


def draw_system_u(nocc_a: int, nocc_b: int, nmo: int, naux: int, seed: int,
                  mix: float = 0.05):
    """Open-shell (unrestricted) system: returns (eps_a, eps_b, B_a, B_b).

    The alpha set is drawn as draw_system(nocc_a, nmo - nocc_a, naux, seed).
    Then, from the same generator: beta energies (nocc_b occupied ~ U[-2.0,
    -0.3], nmo - nocc_b virtual ~ U[0.1, 5.0], each sorted) and a rotation
    U = exp(K) of the orbitals, K antisymmetric with entries ~ N(0, mix^2)
    above the diagonal; B_b^Q = U^T B_a^Q U (alpha and beta orbitals of an
    unrestricted reference span the same space but differ)."""
    from scipy.linalg import expm
    rng = np.random.default_rng(seed)
    eps_a, B_a = draw_system(nocc_a, nmo - nocc_a, naux, seed, rng)
    eps_b = np.concatenate([np.sort(rng.uniform(-2.0, -0.3, size=nocc_b)),
                            np.sort(rng.uniform(0.1, 5.0, size=nmo - nocc_b))])
    K = np.triu(rng.standard_normal((nmo, nmo)) * mix, 1)
    U = expm(K - K.T)
    B_b = np.einsum("pr,Qpq,qs->Qrs", U, B_a, U, optimize=True)
    B_b = 0.5 * (B_b + B_b.transpose(0, 2, 1))
    return eps_a, eps_b, B_a, np.ascontiguousarray(B_b)


def draw_batch_sizes(rng: np.random.Generator):
    """Batched workload: nocc ~ U{10..40}, nvir ~ U{8*nocc..12*nocc}, naux = 3*nvir."""
    nocc = int(rng.integers(10, 41))
    nvir = int(rng.integers(8 * nocc, 12 * nocc + 1))
    return nocc, nvir, 3 * nvir


def make_batch_system(system: int, max_nocc: int | None = None):
    """System `system` of the batched EA-ADC(2) workload (index 5): sizes drawn
    by draw_batch_sizes, then eps and B, all from seed_for(5, system).  Systems
    0..63 are the evaluation batch, 100..299 the training set.  max_nocc caps
    nocc (smaller stand-ins for quick checks; the cap is applied to the drawn
    value, the rest of the recipe is unchanged)."""
    seed = seed_for(5, system)
    rng = np.random.default_rng(seed)
    nocc, nvir, naux = draw_batch_sizes(rng)
    if max_nocc is not None and nocc > max_nocc:
        nvir = int(round(nvir * max_nocc / nocc))
        nocc = max_nocc
        naux = 3 * nvir
    eps, B = draw_system(nocc, nvir, naux, seed, rng)
    return eps, B, (nocc, nvir, naux)


def make_system(key: str, system: int = 0):
    """Inputs of a named workload: returns (eps, B, workload)."""
    w = WORKLOADS[key]
    eps, B = draw_system(w.nocc, w.nvir, w.naux, seed_for(w.index, system))
    return eps, B, w


def small_system(nocc: int, nvir: int, naux: int, seed: int, scale: float = 1.0):
    """A small seeded system for parity tests; `scale` multiplies B."""
    eps, B = draw_system(nocc, nvir, naux, seed)
    return eps, B * scale


def random_vectors(dim: int, nvec: int, seed: int) -> np.ndarray:
    """Seeded trial vectors [nvec][dim] ~ N(0,1)."""
    return np.random.default_rng(seed).standard_normal((nvec, dim))

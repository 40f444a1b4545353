"""The seeded input recipe: the threaded scatter used for large systems gives
exactly the values of the plain per-Q loop (the draws stay in Q order)."""
import numpy as np

from synthetic import draw_system


def test_threaded_draw_matches_plain_loop():
    nocc, nvir, naux, seed = 10, 120, 1200, 77       # above the threading threshold
    n = nocc + nvir
    assert naux * n * n >= (1 << 24)
    eps, B = draw_system(nocc, nvir, naux, seed)
    rng = np.random.default_rng(seed)
    eo = np.sort(rng.uniform(-2.0, -0.3, size=nocc))
    ev = np.sort(rng.uniform(0.1, 5.0, size=nvir))
    assert np.array_equal(eps, np.concatenate([eo, ev]))
    iu, ju = np.triu_indices(n)
    for q in range(naux):
        x = rng.standard_normal(iu.size) * (0.3 * np.exp(-q / 40.0))
        if q % 97 == 0 or q == naux - 1:
            m = np.empty((n, n))
            m[iu, ju] = x
            m[ju, iu] = x
            assert np.array_equal(B[q], m), q
    assert np.array_equal(B, B.transpose(0, 2, 1))

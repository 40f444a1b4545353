"""The host eigensolver of the Davidson projected problem (Householder
tridiagonalisation + implicit QR, csrc/syev_host.hpp), compiled with g++ and
checked against LAPACK (numpy.linalg.eigh): eigenvalues, residuals and
orthonormality on random, graded, degenerate and rank-one matrices."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = r"""
#include "syev_host.hpp"
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
    const long long cap = argc > 1 ? std::atoll(argv[1]) : -1;
    int n;
    while (std::scanf("%d", &n) == 1) {
        std::vector<double> A((size_t)n * n), w(n), S((size_t)n * n);
        for (auto& x : A) if (std::scanf("%lf", &x) != 1) return 2;
        if (!adc::syev_host(n, A.data(), w.data(), S.data(), n, cap)) { std::printf("FAIL\n"); continue; }
        for (double x : w) std::printf("%.17g\n", x);
        for (double x : S) std::printf("%.17g\n", x);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def solver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("syev")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2012_06714_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    return str(exe)


def _matrices():
    rng = np.random.default_rng(5)
    out = []
    for n in (1, 2, 3, 7, 16, 33, 64, 128):
        a = rng.standard_normal((n, n))
        out.append(a + a.T)
        g = np.diag(-1e6 + 1e4 * np.arange(n)) + 1e-3 * (a + a.T)   # graded, nearly diagonal
        out.append(g)
    out.append(np.diag(np.arange(12) % 3).astype(float))               # degenerate, diagonal
    out.append(np.ones((20, 20)))                                      # rank one
    q, _ = np.linalg.qr(rng.standard_normal((24, 24)))
    out.append(q @ np.diag(np.repeat([1.0, 2.0, 2.0 + 1e-13], 8)) @ q.T)   # clusters
    return out


def test_host_eigensolver_matches_lapack(solver):
    mats = _matrices()
    text = "".join(f"{m.shape[0]}\n" + " ".join(f"{x:.17g}" for x in m.ravel()) + "\n" for m in mats)
    res = subprocess.run([solver], input=text, capture_output=True, text=True, check=True)
    vals = res.stdout.split()
    pos = 0
    for a in mats:
        n = a.shape[0]
        assert vals[pos] != "FAIL"
        w = np.array(vals[pos:pos + n], dtype=float)
        S = np.array(vals[pos + n:pos + n + n * n], dtype=float).reshape(n, n)
        pos += n + n * n
        scale = max(np.abs(a).max(), 1e-300)
        ref = np.linalg.eigvalsh(a)
        assert np.all(np.diff(w) >= 0)
        assert np.abs(w - ref).max() <= 1e-13 * n * scale
        assert np.abs(S @ S.T - np.eye(n)).max() <= 1e-13 * n
        assert np.abs(a @ S.T - S.T * w).max() <= 1e-13 * n * scale
    assert pos == len(vals)


def test_host_eigensolver_reports_unconverged_sweeps(solver):
    """With the QR sweep budget set to 0 a matrix that is not already diagonal
    cannot converge: the solver must say so (the Davidson driver then hands
    the projected problem to rocSOLVER), while a diagonal one needs no sweep."""
    rng = np.random.default_rng(9)
    a = rng.standard_normal((6, 6))
    a = a + a.T
    d = np.diag([3.0, 1.0, 2.0])
    text = "".join(f"{m.shape[0]}\n" + " ".join(f"{x:.17g}" for x in m.ravel()) + "\n"
                   for m in (a, d))
    res = subprocess.run([solver, "0"], input=text, capture_output=True, text=True, check=True)
    vals = res.stdout.split()
    assert vals[0] == "FAIL"
    w = np.array(vals[1:4], dtype=float)
    assert np.array_equal(w, [1.0, 2.0, 3.0])

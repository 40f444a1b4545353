// Eigenpairs of a small symmetric matrix on the host: Householder reduction
// to tridiagonal form with the reflections accumulated, then implicit QR
// sweeps with Wilkinson shifts (Golub & Van Loan, "Matrix Computations",
// Sec. 8.3).  Used for the Rayleigh-Ritz problem of the Davidson solver, whose
// projected matrix is assembled on the host anyway.
#pragma once

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>
#include <vector>

namespace adc {

// A: n x n symmetric, row-major (only read).  On success w[k] holds the
// eigenvalues in ascending order and row k of S (n x n, row-major) the unit
// eigenvector of w[k]; the lowest nref eigenvalues are recomputed as Rayleigh
// quotients of their vectors.  Returns false when the QR sweeps do not converge
// within max_sweeps (default 60 n) implicit QR steps.
inline bool syev_host(int n, const double* A, double* w, double* S, int nref = 0,
                      long long max_sweeps = -1) {
    if (n <= 0) return true;
    // Zt holds the accumulated transformation transposed (row k = column k),
    // so that rotations and reflections touch contiguous rows
    std::vector<double> a(A, A + (size_t)n * n), Zt((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n), u(n);
    // ---- tridiagonal form: for column k, one reflection H = I - beta v v^T
    // maps a[k+1.., k] onto a multiple of the first unit vector
    for (int k = 0; k + 2 < n; ++k) {
        double xx = 0.0;
        for (int i = k + 1; i < n; ++i) xx += a[(size_t)i * n + k] * a[(size_t)i * n + k];
        if (xx == 0.0) continue;
        const double xn = std::sqrt(xx);
        const double x0 = a[(size_t)(k + 1) * n + k];
        const double alpha = x0 > 0.0 ? -xn : xn;
        double vv = 0.0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = a[(size_t)i * n + k] - (i == k + 1 ? alpha : 0.0);
            vv += v[i] * v[i];
        }
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // trailing block: H A H = A - v q^T - q v^T, p = beta A v, q = p - (beta/2)(v.p) v
        double vp = 0.0;
        for (int i = k + 1; i < n; ++i) {
            double s = 0.0;
            const double* ai = &a[(size_t)i * n];
            for (int j = k + 1; j < n; ++j) s += ai[j] * v[j];
            p[i] = beta * s;
            vp += v[i] * p[i];
        }
        const double K = 0.5 * beta * vp;
        for (int i = k + 1; i < n; ++i) p[i] -= K * v[i];
        for (int i = k + 1; i < n; ++i) {
            double* ai = &a[(size_t)i * n];
            for (int j = k + 1; j < n; ++j) ai[j] -= v[i] * p[j] + p[i] * v[j];
        }
        a[(size_t)(k + 1) * n + k] = a[(size_t)k * n + k + 1] = alpha;
        for (int i = k + 2; i < n; ++i) a[(size_t)i * n + k] = a[(size_t)k * n + i] = 0.0;
        // Z <- Z H, i.e. Zt <- H Zt: u = Zt^T v, Zt -= beta v u^T
        std::fill(u.begin(), u.end(), 0.0);
        for (int j = k + 1; j < n; ++j) {
            const double* zj = &Zt[(size_t)j * n];
            for (int r = 0; r < n; ++r) u[r] += v[j] * zj[r];
        }
        for (int j = k + 1; j < n; ++j) {
            double* zj = &Zt[(size_t)j * n];
            const double f = beta * v[j];
            for (int r = 0; r < n; ++r) zj[r] -= f * u[r];
        }
    }
    std::vector<double> d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)(i + 1) * n + i];
    // ---- implicit QR on the unreduced trailing block [lo, hi]
    const double eps = DBL_EPSILON;
    int hi = n - 1;
    long long sweeps = 0;
    if (max_sweeps < 0) max_sweeps = 60LL * n;
    while (hi > 0) {
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        if (++sweeps > max_sweeps) return false;
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo])))
            --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        // Wilkinson shift: the eigenvalue of the trailing 2x2 block nearer d[hi]
        const double t = 0.5 * (d[hi - 1] - d[hi]), b = e[hi - 1];
        const double mu = d[hi] - b * b / (t + std::copysign(std::hypot(t, b), t));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // rotation G = [[c, s], [-s, c]] on (k, k+1) with G^T (x, z) = (r, 0)
            const double r = std::hypot(x, z);
            const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : -z / r;
            if (k > lo) e[k - 1] = r;
            const double dk = d[k], dk1 = d[k + 1], ek = e[k];
            d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
            if (k + 1 < hi) {
                z = -s * e[k + 1];          // bulge at (k+2, k)
                e[k + 1] *= c;
                x = e[k];
            }
            double* zk = &Zt[(size_t)k * n];
            double* zk1 = &Zt[(size_t)(k + 1) * n];
            for (int row = 0; row < n; ++row) {
                const double g = zk[row], h = zk1[row];
                zk[row] = c * g - s * h;
                zk1[row] = s * g + c * h;
            }
        }
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int i, int j) { return d[i] < d[j]; });
    // the lowest nref eigenvalues as Rayleigh quotients s^T A s of the computed
    // unit vectors: the QR sweeps leave errors of up to a few hundred ulps of
    // ||A|| on the diagonal, the quotient is accurate to the rounding of the
    // products
    nref = std::min(std::max(nref, 0), n);
    for (int k = 0; k < n; ++k) {
        const double* sk = &Zt[(size_t)ord[k] * n];
        std::copy_n(sk, n, &S[(size_t)k * n]);
        w[k] = d[ord[k]];
        if (k >= nref) continue;
        double q = 0.0, nn = 0.0;
        for (int i = 0; i < n; ++i) {
            double t = 0.0;
            const double* ai = A + (size_t)i * n;
            for (int j = 0; j < n; ++j) t += ai[j] * sk[j];
            q += sk[i] * t;
            nn += sk[i] * sk[i];
        }
        w[k] = q / nn;
    }
    // keep the ascending order (the quotients can only swap values that agree
    // to rounding)
    for (int k = 1; k < nref; ++k)
        for (int j = k; j > 0 && w[j] < w[j - 1]; --j) {
            std::swap(w[j], w[j - 1]);
            std::swap_ranges(&S[(size_t)j * n], &S[(size_t)j * n] + n, &S[(size_t)(j - 1) * n]);
        }
    return true;
}

}  // namespace adc

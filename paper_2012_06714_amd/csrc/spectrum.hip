// Density of states and propagator from the solver's outputs (Sec. II: the
// ADC propagator G(w) = X (w - Omega)^-1 X^T and A(w) = -(1/pi) Im Tr G;
// Sec. IV: the photoelectron spectrum as a sum of Lorentzians of width eta
// weighted by the spectroscopic factors).  Memory-bound elementwise work:
// one thread per output, the roots staged through LDS in chunks.
#include "adc_internal.hpp"

namespace adc {

namespace {

constexpr int CH = 1024;   // roots per LDS chunk
constexpr double INV_PI = 0.31830988618379067154;

// A[k] = (1/pi) sum_mu P_mu eta / ((w_k - e_mu)^2 + eta^2)
__global__ void k_spectral(const double* __restrict__ w, int nw, const double* __restrict__ e,
                           const double* __restrict__ P, int nr, double eta,
                           double* __restrict__ A) {
    __shared__ double se[CH], sp[CH];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double wk = k < nw ? w[k] : 0.0;
    const double eta2 = eta * eta;
    double acc = 0.0;
    for (int m0 = 0; m0 < nr; m0 += CH) {
        const int n = min(CH, nr - m0);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            se[i] = e[m0 + i];
            sp[i] = P[m0 + i];
        }
        __syncthreads();
        for (int i = 0; i < n; ++i) {
            const double d = wk - se[i];
            acc += sp[i] / (d * d + eta2);
        }
    }
    if (k < nw) A[k] = acc * eta * INV_PI;
}

// G[k][p] = sum_mu X[mu][p]^2 / (w_k - e_mu + i eta), stored (re, im)
__global__ void k_prop_diag(const double* __restrict__ w, int nw, const double* __restrict__ e,
                            const double* __restrict__ X, int nr, int norb, double eta,
                            double* __restrict__ G) {
    const long long total = (long long)nw * norb;
    for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(o / norb), p = (int)(o - (long long)k * norb);
        const double wk = w[k];
        double re = 0.0, im = 0.0;
        for (int m = 0; m < nr; ++m) {
            const double x = X[(long long)m * norb + p];
            const double d = wk - e[m];
            const double s = x * x / (d * d + eta * eta);
            re += s * d;
            im -= s * eta;
        }
        G[2 * o] = re;
        G[2 * o + 1] = im;
    }
}

}  // namespace

void spectral_function(hipStream_t st, const double* w, int nw, const double* e, const double* P,
                       int nr, double eta, double* A) {
    hipLaunchKernelGGL(k_spectral, dim3((nw + 255) / 256), dim3(256), 0, st, w, nw, e, P, nr, eta,
                       A);
    ADC_HIP(hipGetLastError());
}

void propagator_diag(hipStream_t st, const double* w, int nw, const double* e, const double* X,
                     int nr, int norb, double eta, double* G) {
    const long long total = (long long)nw * norb;
    long long g = (total + 255) / 256;
    if (g > (1LL << 20)) g = 1LL << 20;
    hipLaunchKernelGGL(k_prop_diag, dim3((unsigned)g), dim3(256), 0, st, w, nw, e, X, nr, norb,
                       eta, G);
    ADC_HIP(hipGetLastError());
}

}  // namespace adc

// Learned Davidson preconditioner: a per-element multilayer perceptron that
// corrects the diagonal preconditioner of the multiroot Davidson solver
// (Sec. III.A, step 4):
//   delta_e = rhat_e q_e (1 + y_e),   rhat = r / rms(r),
//   q_e = 1 / (theta - D_e)  (|theta - D_e| floored at 1e-8),
//   y_e = w3 . tanh(W2 tanh(W1 f_e + b1) + b2) + b3,
// with NF = 7 features f_e (S = max |eps| of the system):
//   (theta - D_e)/S, rhat_e, the three orbital energies of the element / S
//   (EA 2p1h (i,a,b): eps_i, eps_a, eps_b; 1p a: 0, eps_a, 0; IP 2h1p (a,i,j):
//   eps_a, eps_i, eps_j; 1h i: 0, eps_i, 0), theta/S, single-block flag.
// Parameters: one flat FP32 vector W1[256][7], b1[256], W2[256][256], b2[256],
// w3[256], b3.  Training pairs come from the solver's own iterates: target
// t = -e/rms(e) rms(rhat q), e the error of the iterate x against the
// converged eigenvector projected off x; loss 0.5 mean (delta - t)^2; Adam.
//
// Kernels: feature/pair gathers and reductions (HBM-bound), the 256-wide
// hidden layer as a matrix-core GEMM (FP32 for training, BF16 products with
// FP32 sums for inference), tanh/bias/combination elementwise kernels, the
// weight gradients as long-K (split) GEMMs, and the Adam update.
#include "context.hpp"

#include <cmath>
#include <map>
#include <mutex>
#include <string>

namespace adc {

static constexpr int NF = MLP_NF, WD = MLP_WIDTH;
static constexpr long long OFF_W1 = 0, OFF_B1 = OFF_W1 + WD * NF, OFF_W2 = OFF_B1 + WD,
                           OFF_B2 = OFF_W2 + WD * WD, OFF_W3 = OFF_B2 + WD, OFF_B3 = OFF_W3 + WD;
static_assert(OFF_B3 + 1 == MLP_NPARAM, "parameter layout");

static unsigned nblocks(long long n, int bs = 256) {
    long long g = (n + bs - 1) / bs;
    if (g > (1LL << 20)) g = 1LL << 20;
    return (unsigned)(g < 1 ? 1 : g);
}

struct OrbArgs {
    const double *eo, *ev;
    int kind, n1, np;
    double inv_s;
};

// orbital energies (x, p, q) and the single-block flag of element e
__device__ inline void element_orbitals(long long e, const OrbArgs& o, double& ex, double& ep,
                                        double& eq, float& single) {
    const bool ea = o.kind == ADC_EA;
    if (e < o.n1) {
        ex = 0.0;
        ep = ea ? o.ev[e] : o.eo[e];
        eq = 0.0;
        single = 1.f;
        return;
    }
    const long long f = e - o.n1, pp = (long long)o.np * o.np;
    const long long x = f / pp, rem = f - x * pp;
    const int p = (int)(rem / o.np), q = (int)(rem - (long long)p * o.np);
    ex = ea ? o.eo[x] : o.ev[x];
    ep = ea ? o.ev[p] : o.eo[p];
    eq = ea ? o.ev[q] : o.eo[q];
    single = 0.f;
}

__device__ inline double floor_den(double den) {
    if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
    return den;
}

__device__ inline void write_features(float* F, double theta, double D, double rhat, double ex,
                                      double ep, double eq, float single, double inv_s) {
    F[0] = (float)((theta - D) * inv_s);
    F[1] = (float)rhat;
    F[2] = (float)(ex * inv_s);
    F[3] = (float)(ep * inv_s);
    F[4] = (float)(eq * inv_s);
    F[5] = (float)(theta * inv_s);
    F[6] = single;
}

// ---------------------------------------------------------------------------
// reductions: per-block partial sums of up to 5 products, finished on the host
// ---------------------------------------------------------------------------
// sums: 0 x.xs, 1 x.x, 2 xs.xs, 3 r.r, 4 (r q)^2
__global__ void k_pair_sums(const double* __restrict__ x, const double* __restrict__ xs,
                            const double* __restrict__ r, const double* __restrict__ D,
                            double theta, long long n, double* __restrict__ part) {
    double s[5] = {0, 0, 0, 0, 0};
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const double xv = x ? x[e] : 0.0, sv = xs ? xs[e] : 0.0, rv = r[e];
        const double rq = rv / floor_den(theta - D[e]);
        s[0] += xv * sv;
        s[1] += xv * xv;
        s[2] += sv * sv;
        s[3] += rv * rv;
        s[4] += rq * rq;
    }
    __shared__ double red[5][256];
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) part[(long long)blockIdx.x * 5 + k] = red[k][0];
}

static void pair_sums(adc_ctx* c, const double* x, const double* xs, const double* r,
                      double theta, double out[5]) {
    Engine& E = c->E;
    const long long n = c->dim;
    const unsigned nb = (unsigned)std::min<long long>(1024, (n + 255) / 256);
    double* part = (double*)E.scratch.get(40, sizeof(double) * 5 * nb);
    hipLaunchKernelGGL(k_pair_sums, dim3(nb), dim3(256), 0, E.stream, x, xs, r, c->diag.p, theta,
                       n, part);
    ADC_HIP(hipGetLastError());
    std::vector<double> h((size_t)5 * nb);
    ADC_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           E.stream));
    ADC_HIP(hipStreamSynchronize(E.stream));
    for (int k = 0; k < 5; ++k) out[k] = 0.0;
    for (unsigned b = 0; b < nb; ++b)
        for (int k = 0; k < 5; ++k) out[k] += h[(size_t)b * 5 + k];
}

// ---------------------------------------------------------------------------
// training pairs for sampled elements
// ---------------------------------------------------------------------------
struct PairScalars {
    double theta, inv_rms_r, sgn, ex_coef, inv_rms_e, rms_rq;
};

__global__ void k_pairs(const double* __restrict__ x, const double* __restrict__ xs,
                        const double* __restrict__ r, const double* __restrict__ D,
                        const long long* __restrict__ idx, long long nidx, OrbArgs o,
                        PairScalars s, float* __restrict__ F, float* __restrict__ a,
                        float* __restrict__ t) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < nidx;
         j += (long long)gridDim.x * blockDim.x) {
        const long long e = idx[j];
        double ex, ep, eq;
        float single;
        element_orbitals(e, o, ex, ep, eq, single);
        const double rhat = r[e] * s.inv_rms_r;
        const double q = 1.0 / floor_den(s.theta - D[e]);
        write_features(F + j * NF, s.theta, D[e], rhat, ex, ep, eq, single, o.inv_s);
        a[j] = (float)(rhat * q);
        // e_perp = (sgn xs - x) - ex_coef x
        const double err = s.sgn * xs[e] - x[e] - s.ex_coef * x[e];
        t[j] = (float)(-err * s.inv_rms_e * s.rms_rq);
    }
}

void mlp_pairs(adc_ctx* c, const double* x, const double* r, double theta, const double* xstar,
               const long long* idx, long long nidx, float* F, float* a, float* t) {
    Engine& E = c->E;
    const double n = (double)c->dim;
    double s5[5];
    pair_sums(c, x, xstar, r, theta, s5);
    const double dxs = s5[0], xx = s5[1], ss = s5[2], rr = s5[3], rq2 = s5[4];
    ADC_REQUIRE(xx > 0 && ss > 0 && rr > 0, "mlp_pairs: zero vector");
    PairScalars p;
    p.theta = theta;
    p.inv_rms_r = 1.0 / std::sqrt(rr / n);
    p.sgn = dxs < 0 ? -1.0 : 1.0;
    // e = sgn xs - x;  e.x = sgn dxs - xx;  e_perp = e - (e.x / xx) x
    const double ex_dot = p.sgn * dxs - xx;
    p.ex_coef = ex_dot / xx;
    const double ee = ss - 2.0 * p.sgn * dxs + xx;
    const double eperp2 = std::max(ee - ex_dot * ex_dot / xx, 1e-300);
    p.inv_rms_e = 1.0 / std::sqrt(eperp2 / n);
    // rms(rhat q) = rms(r q) / rms(r)
    p.rms_rq = std::sqrt(rq2 / n) * p.inv_rms_r;
    OrbArgs o{c->eo.p, c->ev.p, c->kind, c->n1, (int)c->n2p, 1.0 / c->escale};
    hipLaunchKernelGGL(k_pairs, dim3(nblocks(nidx)), dim3(256), 0, E.stream, x, xstar, r,
                       c->diag.p, idx, nidx, o, p, F, a, t);
    ADC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// H1[e][j] = tanh(sum_f W1[j][f] F[e][f] + b1[j])
__global__ void k_layer1(const float* __restrict__ P, const float* __restrict__ F, long long n,
                         float* __restrict__ H1) {
    __shared__ float w[WD * NF + WD];
    for (int i = threadIdx.x; i < WD * NF + WD; i += blockDim.x) w[i] = P[OFF_W1 + i];
    __syncthreads();
    const long long total = n * WD;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (long long)gridDim.x * blockDim.x) {
        const long long e = g / WD;
        const int j = (int)(g - e * WD);
        const float* f = F + e * NF;
        float s = w[WD * NF + j];
#pragma unroll
        for (int k = 0; k < NF; ++k) s += w[j * NF + k] * f[k];
        H1[g] = tanhf(s);
    }
}

// H[e][j] = tanh(Z[e][j] + b[j])
__global__ void k_bias_tanh(const float* __restrict__ Z, const float* __restrict__ b, long long n,
                            float* __restrict__ H) {
    const long long total = n * WD;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (long long)gridDim.x * blockDim.x)
        H[g] = tanhf(Z[g] + b[g % WD]);
}

// y[e] = w3 . H2[e] + b3: one wave per row, 4 elements per lane
__global__ void k_layer3(const float* __restrict__ P, const float* __restrict__ H2, long long n,
                         float* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nw = ((long long)gridDim.x * blockDim.x) >> 6;
    const float4 w = reinterpret_cast<const float4*>(P + OFF_W3)[lane];
    const float b3 = P[OFF_B3];
    for (long long e = wave; e < n; e += nw) {
        const float4 h = reinterpret_cast<const float4*>(H2 + e * WD)[lane];
        float s = h.x * w.x + h.y * w.y + h.z * w.z + h.w * w.w;
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) y[e] = s + b3;
    }
}

struct Work {
    float *H1, *H2, *Z;
};

static Work work(adc_ctx* c, long long n) {
    Engine& E = c->E;
    Work w;
    w.H1 = (float*)E.scratch.get(41, sizeof(float) * n * WD);
    w.H2 = (float*)E.scratch.get(42, sizeof(float) * n * WD);
    w.Z = (float*)E.scratch.get(43, sizeof(float) * n * WD);
    return w;
}

static void forward(Engine& E, const float* P, const float* F, long long n, bool bf16,
                    const Work& w, float* y) {
    hipLaunchKernelGGL(k_layer1, dim3(nblocks(n * WD)), dim3(256), 0, E.stream, P, F, n, w.H1);
    ADC_HIP(hipGetLastError());
    // Z = H1 W2^T (W2 stored [out][in])
    const bool old = E.bf16;
    E.bf16 = bf16;
    gemm_rm<float>(E, false, true, n, WD, WD, 1.f, w.H1, WD, 0, P + OFF_W2, WD, 0, 0.f, w.Z, WD, 0,
                   1);
    E.bf16 = old;
    hipLaunchKernelGGL(k_bias_tanh, dim3(nblocks(n * WD)), dim3(256), 0, E.stream, w.Z,
                       P + OFF_B2, n, w.H2);
    ADC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_layer3, dim3(nblocks(n * 64)), dim3(256), 0, E.stream, P, w.H2, n, y);
    ADC_HIP(hipGetLastError());
}

void mlp_forward(adc_ctx* c, const float* P, const float* F, long long n, bool bf16, float* y) {
    if (n <= 0) return;
    forward(c->E, P, F, n, bf16, work(c, n), y);
}

// ---------------------------------------------------------------------------
// inference without allocation
// ---------------------------------------------------------------------------
// The hidden activations H1, Z, H2 of up to MLP_NOALLOC_ROWS rows live in this
// file-scope device array (each GPU holds its own copy until the process
// ends).  Its name is only a host-side stand-in: host code uses the address
// hipGetSymbolAddress returns for the current device, looked up once per
// device on the first call there.  Every row of the three activations is
// written before it is read, so nothing needs clearing between calls; calls
// that overlap on one GPU share the array and race.
static __device__ __align__(256) float scratch[MLP_NOALLOC_ROWS * 3 * WD];

static float* noalloc_scratch() {
    static std::mutex mu;
    static std::map<int, float*> ptr;
    int dev = 0;
    ADC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = ptr.find(dev);
    if (it != ptr.end()) return it->second;
    void* p = nullptr;
    ADC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ptr[dev] = static_cast<float*>(p);
    return static_cast<float*>(p);
}

void mlp_forward_noalloc(const float* P, const float* F, long long n, bool bf16, float* y,
                         hipStream_t stream) {
    ADC_REQUIRE(n >= 1 && n <= MLP_NOALLOC_ROWS,
                "adc_mlp_forward_noalloc: n must be 1.." + std::to_string(MLP_NOALLOC_ROWS));
    float* s = noalloc_scratch();
    Engine E;              // stream only: no autotuner trials (they would create events),
    E.stream = stream;     // and the 256-long sums never take the split-K path
    E.autotune = false;
    const Work w{s, s + 2 * MLP_NOALLOC_ROWS * WD, s + MLP_NOALLOC_ROWS * WD};   // H1, H2, Z
    forward(E, P, F, n, bf16, w, y);
}

// ---------------------------------------------------------------------------
// loss and gradient (FP32)
// ---------------------------------------------------------------------------
// diff = a (1 + y) - t;  dy = diff a / n;  per-block partial sums of diff^2
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ a,
                       const float* __restrict__ t, long long n, float* __restrict__ dy,
                       double* __restrict__ part) {
    double s = 0.0;
    const float inv_n = 1.f / (float)n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const float d = a[e] * (1.f + y[e]) - t[e];
        dy[e] = d * a[e] * inv_n;
        s += (double)d * d;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// D2[e][j] = dy[e] w3[j] (1 - H2[e][j]^2)
__global__ void k_back3(const float* __restrict__ P, const float* __restrict__ dy,
                        const float* __restrict__ H2, long long n, float* __restrict__ D2) {
    const long long total = n * WD;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (long long)gridDim.x * blockDim.x) {
        const long long e = g / WD;
        const int j = (int)(g - e * WD);
        const float h = H2[g];
        D2[g] = dy[e] * P[OFF_W3 + j] * (1.f - h * h);
    }
}

// D[g] *= (1 - H[g]^2)
__global__ void k_tanh_grad(const float* __restrict__ H, long long total, float* __restrict__ D) {
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (long long)gridDim.x * blockDim.x) {
        const float h = H[g];
        D[g] *= 1.f - h * h;
    }
}

double mlp_loss_grad(adc_ctx* c, const float* P, const float* F, const float* a, const float* t,
                     long long n, float* G) {
    Engine& E = c->E;
    ADC_REQUIRE(n > 0, "mlp_loss_grad: empty batch");
    const bool old = E.bf16;
    E.bf16 = false;
    Work w = work(c, n);
    float* y = (float*)E.scratch.get(44, sizeof(float) * n);
    float* dy = (float*)E.scratch.get(45, sizeof(float) * n);
    float* ones = (float*)E.scratch.get(46, sizeof(float) * n);
    fill<float>(E, ones, 1.f, (size_t)n);
    forward(c->E, P, F, n, false, w, y);
    const unsigned nb = (unsigned)std::min<long long>(1024, (n + 255) / 256);
    double* part = (double*)E.scratch.get(47, sizeof(double) * nb);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, E.stream, y, a, t, n, dy, part);
    ADC_HIP(hipGetLastError());
    // layer 3: g_w3 = H2^T dy, g_b3 = sum dy
    gemm_rm<float>(E, true, false, WD, 1, n, 1.f, w.H2, WD, 0, dy, 1, 0, 0.f, G + OFF_W3, 1, 0, 1);
    gemm_rm<float>(E, true, false, 1, 1, n, 1.f, dy, 1, 0, ones, 1, 0, 0.f, G + OFF_B3, 1, 0, 1);
    // layer 2: D2 = dy w3 (1 - H2^2) (reuse Z); g_W2 = D2^T H1; g_b2 = D2^T 1
    float* D2 = w.Z;
    hipLaunchKernelGGL(k_back3, dim3(nblocks(n * WD)), dim3(256), 0, E.stream, P, dy, w.H2, n, D2);
    ADC_HIP(hipGetLastError());
    gemm_rm<float>(E, true, false, WD, WD, n, 1.f, D2, WD, 0, w.H1, WD, 0, 0.f, G + OFF_W2, WD, 0,
                   1);
    gemm_rm<float>(E, true, false, WD, 1, n, 1.f, D2, WD, 0, ones, 1, 0, 0.f, G + OFF_B2, 1, 0, 1);
    // layer 1: D1 = (D2 W2) (1 - H1^2) (into H2); g_W1 = D1^T F; g_b1 = D1^T 1
    float* D1 = w.H2;
    gemm_rm<float>(E, false, false, n, WD, WD, 1.f, D2, WD, 0, P + OFF_W2, WD, 0, 0.f, D1, WD, 0,
                   1);
    hipLaunchKernelGGL(k_tanh_grad, dim3(nblocks(n * WD)), dim3(256), 0, E.stream, w.H1, n * WD,
                       D1);
    ADC_HIP(hipGetLastError());
    gemm_rm<float>(E, true, false, WD, NF, n, 1.f, D1, WD, 0, F, NF, 0, 0.f, G + OFF_W1, NF, 0, 1);
    gemm_rm<float>(E, true, false, WD, 1, n, 1.f, D1, WD, 0, ones, 1, 0, 0.f, G + OFF_B1, 1, 0, 1);
    E.bf16 = old;
    std::vector<double> h(nb);
    ADC_HIP(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, E.stream));
    ADC_HIP(hipStreamSynchronize(E.stream));
    double s = 0.0;
    for (double v : h) s += v;
    return 0.5 * s / (double)n;
}

// ---------------------------------------------------------------------------
// Adam
// ---------------------------------------------------------------------------
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

void mlp_adam(adc_ctx* c, float* P, const float* G, float* m, float* v, long long np, int step,
              double lr) {
    ADC_REQUIRE(step >= 1, "mlp_adam: step >= 1");
    const double b1 = 0.9, b2 = 0.999;
    hipLaunchKernelGGL(k_adam, dim3(nblocks(np)), dim3(256), 0, c->E.stream, P, G, m, v, np,
                       (float)lr, (float)b1, (float)b2, 1e-8f, (float)(1.0 - std::pow(b1, step)),
                       (float)(1.0 - std::pow(b2, step)));
    ADC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// inference inside the Davidson solver
// ---------------------------------------------------------------------------
__global__ void k_features(const double* __restrict__ r, const double* __restrict__ D,
                           double theta, double inv_rms, long long e0, long long n, OrbArgs o,
                           float* __restrict__ F) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (long long)gridDim.x * blockDim.x) {
        const long long e = e0 + j;
        double ex, ep, eq;
        float single;
        element_orbitals(e, o, ex, ep, eq, single);
        write_features(F + j * NF, theta, D[e], r[e] * inv_rms, ex, ep, eq, single, o.inv_s);
    }
}

// out[e] = rhat_e q_e (1 + y_e); flags a non-finite result
__global__ void k_combine(const double* __restrict__ r, const double* __restrict__ D,
                          const float* __restrict__ y, double theta, double inv_rms, long long e0,
                          long long n, double* __restrict__ out, int* __restrict__ bad) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (long long)gridDim.x * blockDim.x) {
        const long long e = e0 + j;
        const double v = r[e] * inv_rms / floor_den(theta - D[e]) * (1.0 + (double)y[j]);
        if (!isfinite(v)) *bad = 1;
        out[e] = v;
    }
}

bool mlp_precondition(adc_ctx* c, const double* R, const std::vector<double>& theta,
                      const std::vector<int>& sel, double* Dout) {
    Engine& E = c->E;
    const long long dim = c->dim;
    const long long chunk = std::min<long long>(dim, 1LL << 19);
    float* F = (float*)E.scratch.get(48, sizeof(float) * chunk * NF);
    float* y = (float*)E.scratch.get(49, sizeof(float) * chunk);
    int* bad = (int*)E.scratch.get(50, sizeof(int));
    fill<int>(E, bad, 0, 1);
    Work w = work(c, chunk);
    OrbArgs o{c->eo.p, c->ev.p, c->kind, c->n1, (int)c->n2p, 1.0 / c->escale};
    for (size_t k = 0; k < sel.size(); ++k) {
        const double* r = R + (size_t)sel[k] * dim;
        double s5[5];
        pair_sums(c, nullptr, nullptr, r, theta[sel[k]], s5);
        const double inv_rms = 1.0 / std::sqrt(std::max(s5[3], 1e-300) / (double)dim);
        for (long long e0 = 0; e0 < dim; e0 += chunk) {
            const long long n = std::min(chunk, dim - e0);
            hipLaunchKernelGGL(k_features, dim3(nblocks(n)), dim3(256), 0, E.stream, r,
                               c->diag.p, theta[sel[k]], inv_rms, e0, n, o, F);
            ADC_HIP(hipGetLastError());
            forward(c->E, c->mlp_params.p, F, n, true, w, y);
            hipLaunchKernelGGL(k_combine, dim3(nblocks(n)), dim3(256), 0, E.stream, r, c->diag.p,
                               y, theta[sel[k]], inv_rms, e0, n, Dout + (size_t)k * dim, bad);
            ADC_HIP(hipGetLastError());
        }
    }
    int hbad = 0;
    ADC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, E.stream));
    ADC_HIP(hipStreamSynchronize(E.stream));
    return hbad == 0;
}

}  // namespace adc
